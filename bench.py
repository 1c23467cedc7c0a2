#!/usr/bin/env python
"""Throughput of the TurboReg hot path on one MI355X.

Default workload (the metric's): one synthetic pair per step of the indoor
N = 5000 set (5% inliers, sigma 2 cm, tau = theta = 0.1 m, K1 = 1000, K2 = 2),
a step being one whole registration (compatibility graph, SC2 weights, pivots,
TurboCliques, Kabsch fits, inlier scoring, selection) with inputs resident in
device memory. Other workloads (--workload): indoor_n1000; batch256 (256 pairs
of uneven N in one replayed hipGraph per step); outdoor16 (16 pairs of
N = 20000). Prints one JSON line: registrations/s, per-stage times from HIP
events recorded by the library on its stream (in the layout of the paper's
per-stage table too), the roofline of the dominant kernel, learned vs plain
pivots at equal success rate (32 held-out hard pairs at N = 5000, or the 16
outdoor pairs), the scorer's training throughput (indoor N = 5000), and (indoor
workloads) the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "registrations/s @N=5k; learned vs plain pivots at equal success rate"
PEAK_FP4_TFLOPS = 10100.0   # MI355X dense FP4 MFMA, TFLOP/s (the SC2 product runs on FP4 operands)
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # unpacked float32 vector issue, lane slots / s
COMPAT_SLOTS_PER_PAIR = 22.0   # minimum vector issue slots of one compatibility evaluation
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E, GB/s
WEIGHTS = os.path.join(ROOT, "paper_2507_01439_amd", "weights", "scorer_indoor.bin")
PEAK_FP32_TFLOPS = 157.3    # MI355X float32 rate, vector and MFMA alike (the scorer's training kernels use both)
# Scorer training, per sample (19 -> 64 -> 64 -> 1): multiply-adds of the forward pass (5376), of
# the layer-2 input gradient (4096) and of the weight gradients (5376), two flops each
MLP_TRAIN_FLOP_PER_SAMPLE = 2.0 * (5376 + 4096 + 5376)
# HBM bytes per sample a training step cannot avoid with per-sample activations kept for the
# weight-gradient pass: the 19 bf16 features and the label read twice, four 64-float rows
# (activations and deltas) and two floats (delta and loss) written once and read once
MLP_TRAIN_BYTES_PER_SAMPLE = 2.0 * (38 + 1) + 2.0 * 4 * (4 * 64 + 2)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("graph.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2507_01439_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(name):
    """HBM bytes per launch and the MFMA busy fraction from a committed counter summary ("key:
    value" lines), if it still matches the kernel source; else (None, None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, None
    d = {}
    with open(path) as f:
        for line in f:
            k, sep, v = line.partition(":")
            if sep:
                d[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if d.get("source_hash") != kernel_source_hash():
        return None, None
    try:
        return float(d["hbm_bytes_per_launch"]), float(d.get("mfma_busy_fraction", "nan"))
    except (KeyError, ValueError):
        return None, None


def cpu_baseline(pairs, cfg, budget_s):
    """The oracle (plain C) on a bounded sample of the same workload: its OpenMP build over the
    host's cores (the reported value), and its one-thread build beside it."""
    import oracle

    def timed(threaded, budget):
        done, t0 = 0, time.perf_counter()
        while True:
            p = pairs[done % len(pairs)]
            oracle.register(p.src, p.dst, cfg.tau, cfg.theta, cfg.k1, cfg.k2, threaded=threaded)
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        return done, time.perf_counter() - t0

    n1, t1 = timed(False, budget_s / 3)
    nm, tm = timed(True, 2 * budget_s / 3)
    cores = oracle.threads(True)
    cpu = platform.processor() or platform.machine()
    return {"value": nm / tm, "unit": "registrations/s", "cores": cores, "kind": "oracle",
            "sample": f"{nm} registrations of {min(nm, len(pairs))} distinct pairs of the {cfg.n}-match indoor "
                      f"workload, whole path, OpenMP build, {cores} threads ({cpu}, {os.cpu_count()} cores visible)",
            "single_thread": {"value": n1 / t1, "cores": 1, "sample": f"{n1} registrations, one thread"}}


TABLE7 = {   # the paper's per-stage table: graph construction, pivot-guided search, model estimation
    "graph_construction": ("plan", "compat", "sc2"),
    "pivot_guided_search": ("pivots", "learned", "cliques"),
    "model_estimation": ("kabsch", "score", "select"),
}


def training_rate(torch, minibatch=65536, steps=20, warmup=3):
    """Scorer training throughput: tr_train_step (forward, backward, weight-gradient reduction,
    Adam) on minibatches of features of generated indoor pairs (N ~ U{1000..5000}, inlier ratio
    ~ U[2 %, 30 %], the training recipe), timed with events on the current stream, against the
    float32 vector roof and the HBM roof of its per-sample traffic."""
    from paper_2507_01439_amd import train_scorer
    from paper_2507_01439_amd import turboreg as T
    treg = T.Registrar(max_n=5000, max_batch=32, max_k1=1, max_k2=1)
    try:
        T.tr_scorer_set(treg.h, train_scorer.init_params(1))
        feat, labels = train_scorer.build_features(treg, torch, 32, 32, 5, lambda s: None)
        m = min(minibatch, feat.shape[0])
        xb, yb = feat[:m].contiguous(), labels[:m].contiguous()
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        for _ in range(warmup):
            T.tr_train_step(treg.h, xb, yb, m, 1e-3, loss)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            T.tr_train_step(treg.h, xb, yb, m, 1e-3, loss)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    finally:
        treg.close()
    rate = m / (ms * 1e-3)
    tflops = rate * MLP_TRAIN_FLOP_PER_SAMPLE / 1e12
    gbs = rate * MLP_TRAIN_BYTES_PER_SAMPLE / 1e9
    return {"samples_per_s": rate, "minibatch": m, "ms_per_step": ms, "steps": steps,
            "flop_per_sample": MLP_TRAIN_FLOP_PER_SAMPLE, "achieved_tflops": tflops,
            "fp32_frac": tflops / PEAK_FP32_TFLOPS, "bytes_per_sample": MLP_TRAIN_BYTES_PER_SAMPLE,
            "achieved_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS,
            "kernels": "k_mlp_fwdbwd, k_mlp_wgrad, k_mlp_reduce, k_adam per step"}


def workload(name):
    from paper_2507_01439_amd import synth
    if name in ("indoor_n5000", "indoor_n1000"):
        cfg = synth.CONFIGS[name]
        idx = 1 if name == "indoor_n5000" else 0
        return cfg, [[synth.make_pair(cfg, synth.pair_seed(idx, b))] for b in range(8)]
    if name == "batch256":
        cfgs = synth.batch_configs(256, seed=2, n_lo=500, n_hi=5000)
        cfg = synth.CONFIGS["indoor_n1000"].replace(n=5000, k1=500)
        return cfg, [[synth.make_pair(c, synth.pair_seed(2, b)) for b, c in enumerate(cfgs)]]
    if name == "outdoor16":
        cfg = synth.CONFIGS["outdoor_n20000"]
        return cfg, [[synth.make_pair(cfg, synth.pair_seed(4, b)) for b in range(16)]]
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="indoor_n5000",
                    choices=["indoor_n5000", "indoor_n1000", "batch256", "outdoor16"])
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain comparison at equal success rate (indoor N = 5000 and outdoor16)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--no-training", action="store_true",
                    help="skip the scorer-training throughput (indoor N = 5000 only)")
    ap.add_argument("--concurrent", type=int, default=2, metavar="K",
                    help="also time single-pair registrations spread over K handles on K streams (0: skip)")
    ap.add_argument("--ranking", action="store_true",
                    help="add ranking-based recalls (IN / MSE / MAE ranking) on 32 low-inlier N=5000 pairs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times and sum MIB MiB three times (a "
                         "kernel that reads and writes and one that only reads, of known traffic, for scaling "
                         "hardware byte counters)")
    ap.add_argument("--tuning-cache", metavar="PATH",
                    help="launch configurations: loaded from PATH when it exists (no autotuning then), "
                         "else autotuned and saved to PATH")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not supported "
              "(batches would shard pairs across GPUs, but no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_01439_amd import synth
    from paper_2507_01439_amd import turboreg as T

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.calibrate_copy > 0:
        a = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            c.copy_(a)
        f = a.view(torch.float32)
        for _ in range(3):
            f.sum()
        torch.cuda.synchronize()
        del a, c, f
    cfg, groups = workload(args.workload)
    B = len(groups[0])
    max_n = max(p.src.shape[0] for g in groups for p in g)
    reg = T.Registrar(max_n=max_n, max_batch=B, max_k1=cfg.k1, max_k2=cfg.k2)
    plain = T.params_from_config(cfg)
    prof = T.params_from_config(cfg, flags=T.TR_FLAG_PROFILE)
    dev = []
    for g in groups:
        ns = [p.src.shape[0] for p in g]
        offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
        dev.append(dict(src=torch.from_numpy(np.concatenate([p.src for p in g])).cuda(),
                        dst=torch.from_numpy(np.concatenate([p.dst for p in g])).cuda(),
                        offs=torch.from_numpy(offs).cuda(), n=ns,
                        out=torch.empty(80 * B, dtype=torch.uint8, device="cuda"),
                        mask=torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")))
    G = len(dev)
    side = torch.cuda.Stream()   # default priority; batches replay a captured hipGraph on it

    # launch configuration: the library's autotuner on the first input group (untimed)
    tuned_ms, tuning_source = None, "default"
    if args.tuning_cache and os.path.exists(args.tuning_cache):
        T.tr_tuning_load(reg.h, args.tuning_cache)
        tuning_source = "cache"
    elif not args.no_autotune:
        d = dev[0]
        _, tuned_ms = T.tr_autotune(reg.h, d["src"], d["dst"], None if B == 1 else d["offs"], B,
                                    d["n"][0] if B == 1 else max_n, plain, d["out"], d["mask"])
        torch.cuda.synchronize()
        tuning_source = "autotuned"
        if args.tuning_cache:
            T.tr_tuning_save(reg.h, args.tuning_cache)
    tuning = T.tr_tuning_get(reg.h, max_n, B)

    def step(k, prm):
        d = dev[k % G]
        if B == 1:
            T.tr_register(reg.h, d["src"], d["dst"], d["n"][0], prm, d["out"], d["mask"])
        else:
            T.tr_register_batch(reg.h, d["src"], d["dst"], d["offs"], B, max_n, prm, d["out"], d["mask"])

    # per-stage times: a profiled pass (eager, events recorded on the library's stream)
    for k in range(max(2, args.warmup // 4)):
        step(k, prof)
    torch.cuda.synchronize()
    T.tr_stage_times(reg.h)
    nprof = max(5, min(args.steps, 50))
    for k in range(nprof):
        step(k, prof)
    torch.cuda.synchronize()
    stages = T.tr_stage_times(reg.h)
    # the dominant kernel's launch duration: K steps with only the two events around SC2
    # (recorded by the library on the stream the kernel runs on)
    sc2_only = T.params_from_config(cfg, flags=T.TR_FLAG_PROFILE_SC2)
    for k in range(args.steps):
        step(k, sc2_only)
    torch.cuda.synchronize()
    sc2_ms = T.tr_stage_times(reg.h)["sc2"]

    # timed region: K steps, batches replayed from their hipGraph on the side stream
    with torch.cuda.stream(side):
        for k in range(args.warmup):
            step(k, plain)
        side.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(side)
        for k in range(args.steps):
            step(k, plain)
        ev1.record(side)
        side.synchronize()
        wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    regs = args.steps * B
    ms_per_step = 1000.0 * wall / args.steps

    # serving-style throughput: independent registrations on K handles and K streams, so the
    # latency-bound stages of one overlap the SC2 stage of another (reported beside `value`)
    concurrent = None
    if args.concurrent > 1 and B == 1:
        K = args.concurrent
        handles = [T.Registrar(max_n=max_n, max_batch=1, max_k1=cfg.k1, max_k2=cfg.k2) for _ in range(K)]
        streams = [torch.cuda.Stream() for _ in range(K)]
        bufs = [(torch.empty(80, dtype=torch.uint8, device="cuda"),
                 torch.empty(max_n, dtype=torch.uint8, device="cuda")) for _ in range(K)]
        for hd in handles:
            T.tr_tuning_set(hd.h, max_n, 1, tuning)

        def cstep(k):
            s, d = k % K, dev[k % G]
            with torch.cuda.stream(streams[s]):
                T.tr_register(handles[s].h, d["src"], d["dst"], d["n"][0], plain, bufs[s][0], bufs[s][1])

        for k in range(max(args.warmup, K)):
            cstep(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            cstep(k)
        torch.cuda.synchronize()
        cwall = time.perf_counter() - t0
        concurrent = {"streams": K, "registrations_per_s": args.steps / cwall,
                      "note": "independent single-pair registrations, one handle per stream"}
        for hd in handles:
            hd.close()

    res, ok = [], []
    for g, d in zip(groups, dev):
        r = T.parse_results(d["out"], B)
        res += r
        ok += [synth.success(np.array(x.R).reshape(3, 3), np.array(x.t), p) for x, p in zip(r, g)]

    ns_all = [p.src.shape[0] for p in groups[0]]
    sc2_ops = float(sum(float(n) * n * (n - 1) for n in ns_all))   # per launch: N(N-1)/2 outputs x N MACs x 2
    roof = {"kernel": "k_sc2 (FP4 MFMA, C C^T on the upper triangle, exact in float32)", "bound": "mfma",
            "achieved": sc2_ops / (sc2_ms * 1e-3) / 1e12, "peak": PEAK_FP4_TFLOPS, "unit": "TFLOP/s",
            "traffic": load_counters(f"k_sc2_{args.workload}_traffic.txt")[0],
            "mfma_busy_fraction": load_counters(f"k_sc2_{args.workload}_traffic.txt")[1],
            "avg_launch_us": sc2_ms * 1000.0, "algorithmic_ops_per_launch": sc2_ops}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # k_compat is bound by vector ALU issue: per pair evaluation at least two square roots
    # (quarter rate, 4 issue slots each), six coordinate differences, two squared norms
    # (multiply + two fused multiply-adds each), the length difference and the comparison:
    # 22 lane slots. Peak: 256 CUs x 64 lanes x 2.4 GHz unpacked float32 issue.
    compat_pairs = float(sum(n * (n - 1) / 2.0 for n in ns_all))
    compat_tops = compat_pairs * COMPAT_SLOTS_PER_PAIR / (stages["compat"] * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": regs / wall, "unit": "registrations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+fp4",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs_per_step": B, "n": ns_all[0] if B == 1 else "uneven",
                   "inlier_ratio": cfg.inlier_ratio if B == 1 else "per pair", "sigma_m": cfg.sigma,
                   "tau_m": cfg.tau, "theta_m": cfg.theta, "k1": cfg.k1, "k2": cfg.k2, "pivots": "plain",
                   "graph": "o2graph", "distinct_inputs": G},
        "gpu_event_ms_per_step": gpu_ms / args.steps,
        # stages that launch a kernel (plan: batches only; learned: learned pivots only); the fused
        # hypothesis kernel is split into its phases by in-kernel clock stamps
        "stages_us": {k: round(v * 1000.0, 2) for k, v in stages.items() if v > 0},
        "table7_us": {row: round(sum(stages[k] for k in ks) * 1000.0, 2) for row, ks in TABLE7.items()},
        "dominant_stage": max(stages, key=stages.get),
        "concurrent": concurrent,
        "launch_config": {"source": tuning_source, "sc2_super": tuning.sc2_super,
                          "compat_per_cu": tuning.compat_per_cu, "hyp_ppw": tuning.hyp_ppw,
                          "hyp_per_cu": tuning.hyp_per_cu, "sc2_sparse_cap": tuning.sc2_sparse_cap,
                          "autotune_ms_per_call": tuned_ms},
        "roofline": roof,
        "compat_roofline": {"bound": "alu", "achieved": compat_tops, "peak": PEAK_VALU_TOPS,
                            "unit": "TOP/s (VALU lane slots)", "frac": compat_tops / PEAK_VALU_TOPS,
                            "pair_evaluations_per_launch": compat_pairs},
        "success_rate": float(np.mean(ok)),
        "n_boundary_pairs_mean": float(np.mean([r.n_boundary_pairs for r in res])),
    }
    if args.ranking:
        from paper_2507_01439_amd import diagnostics
        base = synth.CONFIGS["indoor_n5000"]
        rng = np.random.default_rng(17)
        rpairs = [synth.make_pair(base.replace(inlier_ratio=float(q)), synth.pair_seed(8, b))
                  for b, q in enumerate(rng.uniform(0.005, 0.02, size=32))]
        rreg = T.Registrar(max_n=base.n, max_batch=1, max_k1=base.k1, max_k2=2)
        line["ranking_recalls"] = {"pairs": 32, "inlier_ratio": [0.005, 0.02], "k1": base.k1,
                                   "table": {name: diagnostics.ranking_recalls(rreg, torch, rpairs, base.k1,
                                                                               ranking=name)
                                             for name in diagnostics.RANKINGS}}
        rreg.close()
    if not args.no_learned and os.path.exists(WEIGHTS) and args.workload in ("indoor_n5000", "outdoor16"):
        from paper_2507_01439_amd import eval_learned
        if args.workload == "indoor_n5000":   # the hard slice (0.5-1 % inliers)
            lreg = T.Registrar(max_n=5000, max_batch=1, max_k1=1000, max_k2=2)
            _, pairs = eval_learned.held_out(0, 32)
            sweep, ref = (16, 32, 64, 125, 250, 1000), 1000
        else:                                 # the 16 outdoor pairs, scorer trained on indoor pairs
            lreg = T.Registrar(max_n=cfg.n, max_batch=1, max_k1=cfg.k1, max_k2=2)
            pairs = groups[0]
            sweep, ref = (125, 250, 500, 1000, 2500), cfg.k1
        with open(WEIGHTS, "rb") as f:
            T.tr_scorer_load(lreg.h, f.read())
        line["learned_vs_plain"] = eval_learned.compare(lreg, torch, pairs, k1_sweep=sweep, ref_k1=ref)
        lreg.close()
    if not args.no_training and args.workload == "indoor_n5000":
        line["scorer_training"] = training_rate(torch)
    if args.cpu_budget > 0 and args.workload in ("indoor_n5000", "indoor_n1000"):
        line["cpu_baseline"] = cpu_baseline([g[0] for g in groups], cfg, args.cpu_budget)
    reg.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
