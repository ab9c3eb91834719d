#!/usr/bin/env python3
"""Benchmark of the mixed-precision k-means hot path on one MI355X.

Workload: the distance-kernel benchmark shape -- X 1,000,000 x 128 and C
4,096 x 128, FP32 entries N(0,1) -- with the FP16 -> FP64 mixed-precision
assignment (threshold rho~ = 5, equation form).  One step is one Lloyd round
over that input: the fused assignment pass (range check, quantisation, norms,
MFMA cross term, reliability test, FP64 correction, argmin and counters)
followed by the centre update (deterministic segmented FP64 reduction,
division, FP32 rounding, largest centre move, and the pass's SSE in FP64 from
the same read of X).  Inputs are
resident in HBM before timing starts.

Prints ONE JSON line.  Extra keys report the assignment kernel alone, the
plain FP64 direct-formula kernel on the same input, the fallback ratio, the
single-solve Lloyd rate (20,000 x 32, k = 16), the large clustering
(2,000,000 x 64, 1,024 blobs, 50 rounds) in BF16/FP16 -> FP64 (BF16 also
with the hardware-aware threshold), uniform FP32 and plain FP64, the batched segmentation-shaped instances (256 problems, one
batched solve against one solve per problem), serving, and, as
`cpu_baseline`, the CPU oracle timed on a bounded sample of the same
workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_FP16_PEAK_TFLOPS = 2500.0   # MI355X dense FP16 matrix peak
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def serve_run(km, ctx, reqs, arrivals, max_active, budget, keep=False):
    """Submit requests at their arrival times to a server; return per-request
    latency (submit -> done), the wall time from first arrival to last
    completion and, with ``keep``, every request's result."""
    srv = km.Server(ctx, budget, max_active=max_active)
    n = len(reqs)
    t0 = time.perf_counter()
    tickets, t_sub, t_done = [None] * n, [0.0] * n, [None] * n
    nxt, left = 0, n
    while left:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            r = reqs[nxt]
            t_sub[nxt] = time.perf_counter() - t0
            tickets[nxt] = srv.submit(r.X, r.C0, r.iters)
            nxt += 1
        for i in range(nxt):
            if t_done[i] is None:
                rc = srv.poll(tickets[i], 0)
                if rc != 1:
                    if rc != 0:
                        raise RuntimeError("served request %d failed: %d" % (i, rc))
                    t_done[i] = time.perf_counter() - t0
                    left -= 1
        time.sleep(0.0002)
    results = [srv.result(t) for t in tickets] if keep else None
    srv.close()
    lat = [t_done[i] - t_sub[i] for i in range(n)]
    return lat, max(t_done) - min(t_sub), results


def serve_bench(km, ctx, count, seed):
    """Continuous batching vs one solve at a time on Poisson arrivals of
    k-means requests (n log-uniform in [1e3, 1e6], d in {3,16,64,128}, k in
    {8..512}, 30 rounds each, FP16 -> FP64) at 0.5, 1.0 and 1.5 times the
    measured one-at-a-time capacity.  At load 1.0 every served result is
    compared bit for bit with the same request solved one at a time (the
    oracle checks of served results are in the GPU test suite)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import workloads as W
    reqs = W.request_stream(count, 1.0, seed)
    log("serving: generating %d requests" % count)
    with ThreadPoolExecutor(16) as ex:
        list(ex.map(lambda r: r.materialize(), reqs))
    budget = 64 << 30
    # one-at-a-time capacity: back-to-back solves through a single-slot server
    lat1, wall1, _ = serve_run(km, ctx, reqs, [0.0] * count, 1, budget)
    mu1 = count / wall1
    log("serving: one-at-a-time capacity %.1f solves/s" % mu1)
    g = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(g.exponential(1.0 / mu1, size=count))
    arrivals -= arrivals[0]
    out = {"requests": count, "one_at_a_time_capacity_per_s": mu1,
           "points": int(sum(r.n for r in reqs)), "rounds_per_request": reqs[0].iters}
    kept = {}
    for load in (0.5, 1.0, 1.5):
        arr = list(arrivals / load)
        res = {"arrival_rate_per_s": mu1 * load}
        for name, slots in (("one_at_a_time", 1), ("continuous_batching", 64)):
            lat, wall, rs = serve_run(km, ctx, reqs, arr, slots, budget, keep=(load == 1.0))
            if rs is not None:
                kept[name] = rs
            res[name] = {"solves_per_s": count / wall,
                         "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
                         "p99_latency_ms": 1e3 * float(np.percentile(lat, 99))}
            log("serving: load %.1f %s: %.1f solves/s, p50 %.1f ms, p99 %.1f ms" % (
                load, name, res[name]["solves_per_s"], res[name]["p50_latency_ms"],
                res[name]["p99_latency_ms"]))
        out["load_%.1f" % load] = res
    a, b = kept["one_at_a_time"], kept["continuous_batching"]
    same = sum(1 for x, y in zip(a, b)
               if np.array_equal(x["labels"], y["labels"]) and np.array_equal(x["C"], y["C"])
               and np.array_equal(x["sse_hist"], y["sse_hist"], equal_nan=True))
    out["identical_to_one_at_a_time"] = same
    out["oracle_checks"] = "tests/test_gpu_server.py (served request stream against the oracle)"
    return out


KERNEL_SOURCES = ("paper_2407_12208_amd/csrc/km_assign.hip",
                  "paper_2407_12208_amd/csrc/km_device.hpp",
                  "paper_2407_12208_amd/csrc/km_internal.hpp")
TRAFFIC_RECORD = "profiles/k_assign_pipe_fp16_n1e6_d128_k4096_hbm_traffic.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per assignment launch from the committed counter record
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for a
    plain copy of known size), or None when the record is missing or was
    taken on different kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_RECORD)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                key, val = line[2:].split(":", 1)
                rec[key.strip()] = val.strip().strip("`")
    try:
        if rec.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_ms(km, ctx, X, C, prec, reps=3):
    """Median duration (ms) of the assignment kernel of `reps` passes, from
    the library's own events on the launch stream."""
    km.kmeans_assign(ctx, X, C, prec, stats=False)  # workspace and warm-up
    km.kmeans_timing_enable(ctx, True)
    for _ in range(reps):
        km.kmeans_assign(ctx, X, C, prec, stats=False)
    t = km.kmeans_timing_read(ctx)
    km.kmeans_timing_enable(ctx, False)
    import numpy as np
    return float(np.median(t))


def variant_table(km, ctx, torch, np, X, C, Xh, Ch, variants, sample_rows=16384, seed=7):
    """For each precision variant: assignment-kernel time on the whole input,
    the fraction of pairs corrected (eq:eta) and the relative error of the
    per-pair values against the FP64 direct formula on a seeded sample of
    rows against all centres (values materialised by kmeans_pairwise, the
    same arithmetic; reference: the plain FP64 direct-formula kernel on the
    same rows, whose values the GPU tests pin to the CPU oracle)."""
    n, d = X.shape
    k = C.shape[0]
    rows = np.sort(np.random.default_rng(seed).choice(n, size=min(sample_rows, n), replace=False))
    Xs = X[torch.from_numpy(rows).cuda()].contiguous()
    R, _ = km.kmeans_pairwise(ctx, Xs, C, km.Precision(km.KM_EXACT64))
    ref = R.cpu().numpy().astype(np.float64)
    del R
    out = {}
    for name, pr in variants:
        ms = kernel_ms(km, ctx, X, C, pr)
        _, _, _, st = km.kmeans_assign(ctx, X, C, pr, stats=True)
        D, _ = km.kmeans_pairwise(ctx, Xs, C, pr)
        Dh = D.cpu().numpy().astype(np.float64)
        del D
        rel = np.abs(Dh - ref) / np.maximum(ref, 1e-300)
        out[name] = {"kernel_ms": ms, "pairs_per_s": float(n) * k / (ms * 1e-3),
                     "eta": st["n_corrected"] / max(st["n_pairs"], 1),
                     "alpha_used": st["alpha_used"],
                     "max_rel_err_vs_fp64": float(rel.max()),
                     "median_rel_err_vs_fp64": float(np.median(rel))}
        log("variant %s: %.3f ms, eta %.3g, max rel err %.3g" % (
            name, ms, out[name]["eta"], out[name]["max_rel_err_vs_fp64"]))
    out["sample"] = "%d seeded rows x all %d centres" % (len(rows), k)
    return out


def dist_variants(km, ctx, torch, W, np, X, C, Xh, Ch):
    """The distance benchmark's precision variants (full tile + argmin) on
    the N(0,1) input and on the cancellation-prone input (every coordinate
    1e3 + 1e-2 z)."""
    P = km.Precision
    variants = (("fp16_fp64", P(km.KM_LOW_FP16)),
                ("fp16_fp64_alg_alpha", P(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_ALG)),
                ("bf16_fp64", P(km.KM_LOW_BF16)),
                ("bf16_fp64_hw_alpha", P(km.KM_LOW_BF16, km.KM_ALPHA_HW)),
                ("fp32_fp64", P(km.KM_LOW_FP32)),
                ("fp16_uniform", P(km.KM_LOW_FP16, km.KM_ALPHA_NONE)),
                ("bf16_uniform", P(km.KM_LOW_BF16, km.KM_ALPHA_NONE)),
                ("fp32_uniform", P(km.KM_LOW_FP32, km.KM_ALPHA_NONE)),
                # other fallback precisions (uniform rule and FP32 correction)
                ("fp16_fp32", P(km.KM_LOW_FP16, high=km.KM_HIGH_FP32)),
                ("bf16_fp32", P(km.KM_LOW_BF16, high=km.KM_HIGH_FP32)),
                ("fp16_fp16", P(km.KM_LOW_FP16, high=km.KM_HIGH_LOW)),
                ("bf16_bf16", P(km.KM_LOW_BF16, high=km.KM_HIGH_LOW)),
                ("fp32_fp32", P(km.KM_LOW_FP32, high=km.KM_HIGH_LOW)),
                ("fp64_direct", P(km.KM_EXACT64)))
    out = {"normal": variant_table(km, ctx, torch, np, X, C, Xh, Ch, variants)}
    cfg = W.DIST_BENCH
    log("cancellation variant: generating %d x %d" % (cfg["n"], cfg["d"]))
    Xc, Cc = W.cancellation_pair(cfg["n"], cfg["k"], cfg["d"], cfg["seed"])
    Xcd = torch.from_numpy(Xc).cuda()
    Ccd = torch.from_numpy(Cc).cuda()
    cvariants = tuple(v for v in variants if v[0] in ("fp16_fp64", "bf16_fp64", "fp16_uniform",
                                                      "bf16_uniform", "fp32_uniform", "fp16_fp32",
                                                      "bf16_fp32", "fp16_fp16", "bf16_bf16",
                                                      "fp32_fp32", "fp64_direct"))
    out["cancellation"] = variant_table(km, ctx, torch, np, Xcd, Ccd, Xc, Cc, cvariants)
    del Xcd, Ccd
    return out


def large_bench(km, ctx, torch, W, np):
    """Large clustering: 2,000,000 x 64 points from 1,024 blobs (centres
    U[-50,50]^64, per-blob std log-uniform in [0.1, 2]), 50 Lloyd rounds and
    the final pass per variant, from the same initial centres."""
    cfg = W.LLOYD_LARGE
    log("large clustering: generating %d x %d, %d blobs" % (cfg["n"], cfg["d"], cfg["k"]))
    X, _, _ = W.blobs(cfg["n"], cfg["d"], cfg["k"], cfg["seed"], center_box=(-50, 50),
                      std_range=(0.1, 2.0))
    C0 = W.init_centroids(X, cfg["k"], cfg["init_seed"])
    Xd = torch.from_numpy(X).cuda()
    del X
    iters = cfg["iters"]
    out = {"n": cfg["n"], "d": cfg["d"], "k": cfg["k"], "rounds": iters}
    variants = (("bf16_fp64", km.Precision(km.KM_LOW_BF16)),
                ("bf16_fp64_hw_alpha", km.Precision(km.KM_LOW_BF16, km.KM_ALPHA_HW)),
                ("fp16_fp64", km.Precision(km.KM_LOW_FP16)),
                ("fp32_uniform", km.Precision(km.KM_LOW_FP32, km.KM_ALPHA_NONE)),
                ("fp64_direct", km.Precision(km.KM_EXACT64)))
    for name, pr in variants:
        C = torch.from_numpy(C0).cuda()
        km.kmeans_lloyd(ctx, Xd, C, 1, prec=pr, stats=False, sync=True)  # workspace
        C.copy_(torch.from_numpy(C0).cuda())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, hist, st = km.kmeans_lloyd(ctx, Xd, C, iters, prec=pr, sse_hist=True,
                                            stats=True, sync=True)
        dt = time.perf_counter() - t0
        out[name] = {"rounds_per_s": iters / dt, "ms_per_round": 1e3 * dt / (iters + 1),
                     "eta": st["n_corrected"] / max(st["n_pairs"], 1),
                     "final_sse": float(hist[-1].item())}
        log("large %s: %.3f ms per round, eta %.3g" % (name, out[name]["ms_per_round"],
                                                         out[name]["eta"]))
    # precision schedule: uniform FP16 while a round lowers the SSE by at
    # least 1e-3 of it (at most 40 rounds), then FP16 -> FP64
    C = torch.from_numpy(C0).cuda()
    uni = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_NONE)
    late = km.Precision(km.KM_LOW_FP16)
    km.kmeans_lloyd_schedule(ctx, Xd, C, 1, uni, late, 1e-3, 40, stats=False, sync=True)
    C.copy_(torch.from_numpy(C0).cuda())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, hist, st, sw = km.kmeans_lloyd_schedule(ctx, Xd, C, iters, uni, late, 1e-3, 40,
                                                     sse_hist=True, stats=True, sync=True)
    dt = time.perf_counter() - t0
    out["fp16_schedule"] = {"rounds_per_s": iters / dt, "ms_per_round": 1e3 * dt / (iters + 1),
                            "eta": st["n_corrected"] / max(st["n_pairs"], 1),
                            "final_sse": float(hist[-1].item()), "switch_round": sw,
                            "rule": "uniform FP16 while the round's SSE falls by >= 1e-3 of it "
                                    "(<= 40 rounds), then FP16 -> FP64"}
    log("large fp16_schedule: %.3f ms per round, switch at round %d" % (
        out["fp16_schedule"]["ms_per_round"], sw))
    out["speedup_fp16_fp64_vs_fp64_direct"] = (out["fp16_fp64"]["rounds_per_s"] /
                                               out["fp64_direct"]["rounds_per_s"])
    out["speedup_bf16_hw_alpha_vs_fp64_direct"] = (out["bf16_fp64_hw_alpha"]["rounds_per_s"] /
                                                   out["fp64_direct"]["rounds_per_s"])
    return out


def batch_bench(km, ctx, torch, W, np, count=256, iters=30):
    """Batched segmentation-shaped instances: `count` problems (n = H*W
    pixels, H, W ~ U{128..1024}, d = 5 features, k ~ U{4..64}), `iters` rounds
    each, FP16 -> FP64: one batched solve against one Lloyd call per problem
    on the same inputs.  Labels of the two runs are compared."""
    log("batched: generating %d segmentation-shaped instances" % count)
    insts = W.segmentation_batch(count, 3004)
    Xs = [torch.from_numpy(b["X"]).cuda() for b in insts]
    C0s = [torch.from_numpy(b["C0"]).cuda() for b in insts]
    total_n = sum(b["X"].shape[0] for b in insts)
    d = insts[0]["X"].shape[1]
    del insts
    prec = km.Precision(km.KM_LOW_FP16)

    def batched(round_launch=False):
        items = [km.BatchItem(X=X, C=C0.clone(), max_iter=iters) for X, C0 in zip(Xs, C0s)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        km.kmeans_solve_batch(ctx, items, prec, with_sse=False, round_launch=round_launch)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, [it.labels for it in items]

    def one_by_one():
        Cs = [C0.clone() for C0 in C0s]
        labs = [torch.empty(X.shape[0], dtype=torch.int32, device="cuda") for X in Xs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for X, C, lab in zip(Xs, Cs, labs):
            km.kmeans_lloyd(ctx, X, C, iters, prec=prec, labels=lab, stats=False)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, labs

    batched()
    one_by_one()
    tb, lb = batched()
    ts, ls = one_by_one()
    same = all(bool(torch.equal(a, b)) for a, b in zip(lb, ls))
    # the same batch with every problem's rounds in persistent launches
    batched(round_launch=True)
    tp, lp = batched(round_launch=True)
    same_p = all(bool(torch.equal(a, b)) for a, b in zip(lp, ls))
    passes = iters + 1
    # algorithmic bytes of an assignment pass: read X once, write the labels;
    # the rate below divides every pass's bytes by the whole batched solve
    # (centre updates included), not by the assignment kernels alone
    alg_bytes = float(total_n) * (4 * d + 4) * passes
    out = {"problems": count, "points": total_n, "d": d, "rounds": iters,
           "batched_s": tb, "one_by_one_s": ts, "speedup": ts / tb,
           "batched_solves_per_s": count / tb, "one_by_one_solves_per_s": count / ts,
           "labels_identical": same,
           "batched_round_launch_s": tp, "round_launch_labels_identical": same_p,
           "batched_assign_bytes_GBps": alg_bytes / tb / 1e9,
           "batched_frac_of_hbm_peak": alg_bytes / tb / 1e9 / HBM_PEAK_GBS,
           # the sweep-length tuner's choice for this launch (made by the
           # first, untimed batched solve and reused by the timed one)
           "tuner_cache": km.kmeans_tune_dump(ctx).strip()}
    log("batched: %.1f ms batched, %.1f ms one by one, labels identical %s" %
        (1e3 * tb, 1e3 * ts, same))
    # segmentation fidelity (the paper's Diff): labels of each variant against
    # the plain FP64 solve of the same instances, after the best one-to-one
    # matching of cluster ids, on the first 16 instances
    P = km.Precision
    m = min(16, count)
    ref = None
    fid = {}
    for name, pr in (("fp64_direct", P(km.KM_EXACT64)), ("fp16_fp64", prec),
                     ("fp16_uniform", P(km.KM_LOW_FP16, km.KM_ALPHA_NONE)),
                     ("bf16_uniform", P(km.KM_LOW_BF16, km.KM_ALPHA_NONE)),
                     ("fp32_uniform", P(km.KM_LOW_FP32, km.KM_ALPHA_NONE))):
        items = [km.BatchItem(X=X, C=C0.clone(), max_iter=iters) for X, C0 in zip(Xs[:m], C0s[:m])]
        km.kmeans_solve_batch(ctx, items, pr, with_sse=False)
        labs = [it.labels.cpu().numpy() for it in items]
        if ref is None:
            ref = labs
            continue
        diffs = [km.kmeans_label_diff(a, b) for a, b in zip(labs, ref)]
        fid[name] = {"mean_diff_pct": 100.0 * float(np.mean(diffs)),
                     "max_diff_pct": 100.0 * float(np.max(diffs))}
    fid["reference"] = "fp64_direct, %d instances, %d rounds" % (m, iters)
    out["segmentation_diff_vs_fp64"] = fid
    log("batched: Diff vs FP64 %s" % {k: round(v["mean_diff_pct"], 3) for k, v in fid.items()
                                      if isinstance(v, dict)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra measurements")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the precision-variant table of the distance benchmark")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large-clustering measurement")
    ap.add_argument("--batch-problems", type=int, default=256,
                    help="problems in the batched measurement (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=500,
                    help="requests in the serving measurement (0 = skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the hot path would shard rows of X across GPUs; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2407_12208_amd as km
    import workloads as W

    cfg = W.DIST_BENCH
    n, d, k = cfg["n"], cfg["d"], cfg["k"]
    log("generating X %dx%d and C %dx%d (seed %d)" % (n, d, k, d, cfg["seed"]))
    Xh, Ch = W.gaussian_pair(n, k, d, cfg["seed"])
    X = torch.from_numpy(Xh).cuda()
    Ca = torch.from_numpy(Ch).cuda()
    Cb = torch.empty_like(Ca)
    labels = torch.zeros(n, dtype=torch.int32, device="cuda")
    shift = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx = km.Context(0)
    prec = km.Precision(km.KM_LOW_FP16, km.KM_ALPHA_PAPER_EQ, 5.0)
    stream = torch.cuda.current_stream()

    sse = torch.empty(1, dtype=torch.float64, device="cuda")

    def step(c_in, c_out):
        # the pass's SSE is taken by the update, which reads every point's
        # row against the centre it was assigned to
        # labels still holds the previous round's assignment: it seeds the
        # search (Lloyd rounds do the same; results are unchanged)
        km.kmeans_assign(ctx, X, c_in, prec, labels=labels, stats=False, stream=stream,
                         labels_hint=True)
        km.kmeans_update(ctx, X, labels, c_in, C_new=c_out, shift=shift, sse=sse, stream=stream)

    bufs = [Ca, Cb]
    for i in range(args.warmup):
        step(bufs[i & 1], bufs[(i + 1) & 1])
    torch.cuda.synchronize()
    km.kmeans_timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(bufs[(args.warmup + i) & 1], bufs[(args.warmup + i + 1) & 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = km.kmeans_timing_read(ctx)
    km.kmeans_timing_enable(ctx, False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    pairs = float(n) * k
    value = pairs * args.steps / elapsed
    kern_avg_ms = float(np.mean(kern_ms)) if kern_ms else float("nan")
    flops = 2.0 * n * k * d
    achieved = flops / (kern_avg_ms * 1e-3) / 1e12
    log("step %.3f ms, assign kernel %.3f ms (%d launches), %.1f TFLOP/s" %
        (ms_per_step, kern_avg_ms, len(kern_ms), achieved))

    out = {
        "metric": "assign distance-pairs/s & Lloyd iters/s vs FP64 GPU baseline; p50/p99 solve latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16+f64",
        "data": "synthetic",
        "config": {"workload": "distance-kernel benchmark: X 1e6x128, C 4096x128, N(0,1) FP32; "
                               "one Lloyd round (mixed FP16->FP64 assign + centre update)",
                   "n": n, "d": d, "k": k, "low": "fp16", "high": "fp64",
                   "alpha_form": "equation (2 rho gamma)", "rho": 5.0},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_FP16_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "k_assign_pipe<LowF16,128,2,true,false>",
                     "kernel_avg_ms": kern_avg_ms,
                     "algorithmic_flops_per_launch": flops},
    }

    if not args.no_extra:
        extra = {}
        # fallback ratio and SSE of one pass (stats force a wait)
        _, _, _, st = km.kmeans_assign(ctx, X, Ca, prec, labels=labels, stats=True)
        extra["eta"] = st["n_corrected"] / st["n_pairs"]
        extra["alpha_used"] = st["alpha_used"]
        extra["assign_kernel_pairs_per_s"] = pairs / (kern_avg_ms * 1e-3)
        # plain FP64 direct-formula kernel on the same input
        p64 = km.Precision(km.KM_EXACT64)
        km.kmeans_timing_enable(ctx, True)
        for _ in range(3):
            km.kmeans_assign(ctx, X, Ca, p64, labels=labels, stats=False)
        t64 = km.kmeans_timing_read(ctx)
        km.kmeans_timing_enable(ctx, False)
        ms64 = float(np.median(t64))
        extra["fp64_direct_kernel_ms"] = ms64
        extra["fp64_direct_pairs_per_s"] = pairs / (ms64 * 1e-3)
        extra["speedup_assign_vs_fp64_direct"] = ms64 / kern_avg_ms
        extra["fp64_direct_frac_of_fp64_peak"] = (3.0 * n * k * d / (ms64 * 1e-3) / 1e12) / FP64_PEAK_TFLOPS
        if not args.no_variants:
            # the timed rounds moved Ca: the variants use the generated centres
            extra["distance_variants"] = dist_variants(km, ctx, torch, W, np, X,
                                                       torch.from_numpy(Ch).cuda(), Xh, Ch)
        # single Lloyd solve: 20,000 x 32, 16 blobs, 20 rounds + final pass
        cs = W.LLOYD_SMALL
        Xs, _, _ = W.blobs(cs["n"], cs["d"], cs["k"], cs["seed"])
        C0 = W.init_centroids(Xs, cs["k"], cs["init_seed"])
        Xs_d = torch.from_numpy(Xs).cuda()
        res = {}
        C0_d = torch.from_numpy(C0).cuda()
        for name, pr, persistent in (("mixed_fp16_fp64", prec, False),
                                     ("mixed_fp16_fp64_round_launch", prec, True),
                                     ("fp64_direct", p64, False)):
            Cs = C0_d.clone()
            km.kmeans_lloyd(ctx, Xs_d, Cs, cs["iters"], prec=pr, stats=False,
                            round_launch=persistent)
            torch.cuda.synchronize()
            reps = 20
            ts = time.perf_counter()
            for _ in range(reps):
                Cs.copy_(C0_d)
                km.kmeans_lloyd(ctx, Xs_d, Cs, cs["iters"], prec=pr, stats=False,
                                round_launch=persistent)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - ts) / reps
            res[name] = cs["iters"] / dt
        extra["lloyd_small_iters_per_s"] = res["mixed_fp16_fp64"]
        extra["lloyd_small_iters_per_s_round_launch"] = res["mixed_fp16_fp64_round_launch"]
        extra["lloyd_small_iters_per_s_fp64_direct"] = res["fp64_direct"]
        extra["lloyd_small_speedup_vs_fp64_direct"] = res["mixed_fp16_fp64"] / res["fp64_direct"]
        if not args.no_large:
            extra["large_clustering"] = large_bench(km, ctx, torch, W, np)
        if args.batch_problems > 0:
            extra["batched_segmentation"] = batch_bench(km, ctx, torch, W, np,
                                                        count=args.batch_problems)
        if args.serve_requests > 0:
            extra["serving"] = serve_bench(km, ctx, args.serve_requests, 3005)
        out["extra"] = extra
        log("extra: %s" % json.dumps(extra))

    if args.calib_copy_mib > 0:
        # one elementwise kernel that reads and writes `nbytes` each: the
        # reference for the HBM byte counters
        nbytes = args.calib_copy_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nbytes

    if not args.no_cpu:
        import oracle
        threads = oracle.num_threads()
        g = np.random.default_rng(4)
        m = 64
        rows = np.sort(g.choice(n, size=m, replace=False))
        ts = time.perf_counter()
        oracle.assign(Xh[rows], Ch)
        dt = time.perf_counter() - ts
        m = int(min(n, max(64, m * args.cpu_seconds / max(dt, 1e-3))))
        rows = np.sort(g.choice(n, size=m, replace=False))
        ts = time.perf_counter()
        oracle.assign(Xh[rows], Ch)
        dt = time.perf_counter() - ts
        out["cpu_baseline"] = {
            "value": float(m) * k / dt, "unit": "pairs/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d random rows of X against all %d centres (FP64 direct formula, "
                      "exact argmin), %.1f s" % (m, k, dt)}
        log("cpu oracle: %d rows in %.2f s on %d threads" % (m, dt, threads))

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
