"""Benchmark: Flowtree (query, doc) pairs/s on one MI355X, batched vs plain.

Workload (the batched-uneven configuration): the text-shaped ground space
(V = 100k points in R^300, L2-normalised 200-cluster mixture), 1M dataset
distributions and 4096 queries whose support sizes follow P(m) ~ m^-1.1 on
5..500, words drawn Zipf(1.1).  One step is the whole hot path for the 4096
queries: Quadtree prune against all 1M docs to the top 1000, then the batched
Flowtree rerank of those 4096 x 1000 pairs to the top 20.

value = Flowtree pairs of the step / step time (the prune included).
The plain one-launch-per-query Flowtree stage is timed on the same
candidates afterwards and reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|batched_v1m|text|image|tiny|exhaustive]
       [--no-cpu-baseline] [--no-plain]
       python bench.py --workload act [--act-cand C] [--act-iters I]   (the R-WMD / ACT stage after
                                                              Flowtree: Quadtree 1000 -> Flowtree C -> ACT-I top-20)
       python bench.py --workload sinkhorn [--act-cand C] [--sk-iters I]   (Sinkhorn-I in place of ACT)
       python bench.py --workload exact [--act-cand C]   (exact W1 of the best C by Flowtree, C = 20)
       python bench.py --workload pipeline   (the four stages end to end, queries/s: Quadtree 1000 ->
                                              Flowtree 100 -> ACT-1 5 -> exact W1 top-1)
       python bench.py --workload random_model [--reps R]   (the Section 3.2 experiment: success
                                                              rate of recovering the planted nearest
                                                              neighbour, Quadtree vs Flowtree, vs N)
       python bench.py --workload recall [--trees T]   (recall@m of Quadtree, eps-weighted Quadtree
                                                 and Flowtree against the exact W1 nearest neighbour, mean
                                                 and std over T random shifts; R-WMD, ACT-1 and
                                                 Sinkhorn-1 beside them)
       python bench.py --workload grad   (forward + backward of the Flowtree cost of 256 pairs on
                                          V = 50k points in R^300, tree and flow pattern frozen)
       python bench.py --calibrate-copy BYTES   (a plain device copy of BYTES, five times: the
                                                 reference for the HBM byte counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

# HBM bytes of one launch of the persistent Flowtree graph per workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy
# (profiles/flowtree_quadtree_batched_hbm_traffic.md, profiles/flowtree_exhaustive_hbm_traffic.md),
# valid while the kernel sources hash to TRAFFIC_SOURCES_SHA1.
TRAFFIC_BYTES = {"batched": 2.7755e+11, "batched_v1m": 4.1655e+11, "exhaustive": 3.7551e+12}
TRAFFIC_SOURCES = ("paper_1910_04126_amd/csrc/flow.h", "paper_1910_04126_amd/csrc/flowtree.hip",
                   "paper_1910_04126_amd/csrc/wave.h", "paper_1910_04126_amd/csrc/common.h")
TRAFFIC_SOURCES_SHA1 = "4c387ec6d488da7f3e0d48b278d4be487d7e8169"


def measured_traffic(workload):
    """The counted bytes when they were taken on this workload and these
    kernel sources, else None."""
    if workload not in TRAFFIC_BYTES:
        return None
    return TRAFFIC_BYTES[workload] if _sources_sha1(TRAFFIC_SOURCES) == TRAFFIC_SOURCES_SHA1 else None


# Counters of the Quadtree prune stage per workload (two query chunks per
# step: k_qt_post ranks, k_topk_window selects), from rocprofv3 --pmc runs
# (profiles/quadtree_prune_batched_counters.md), valid while the prune
# sources hash to PRUNE_SOURCES_SHA1: HBM bytes per step (FETCH_SIZE and
# WRITE_SIZE scaled by the 1 GiB copy), and the ranking kernel's LDS active
# share of cycles, bank-conflict share of LDS cycles, VALU issue against the
# 1.7 per CU-cycle that a VALU-only probe reaches, and L2 hit rate.
PRUNE_COUNTERS = {"batched": {"bytes": 8.4245e+10, "lds_busy": 0.44, "lds_bank_conflict": 0.44,
                              "valu_issue": 0.45, "l2_hit": 0.86}}
PRUNE_SOURCES = ("paper_1910_04126_amd/csrc/quadtree.hip", "paper_1910_04126_amd/csrc/select.hip",
                 "paper_1910_04126_amd/csrc/wave.h", "paper_1910_04126_amd/csrc/common.h")
PRUNE_SOURCES_SHA1 = "8d732dce72eb83c73a589d17fa571f7117083ef4"


def _sources_sha1(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def prune_roofline(workload, stage_ms, n_q, n_docs):
    """The prune stage against the HBM peak: the bytes every pair must move
    with materialised keys (a 4-byte key written, then read by the select),
    and, when taken on these sources, the counted HBM bytes and the ranking
    kernel's counters that name its bound (LDS atomics and L2 latency)."""
    alg = 8.0 * n_q * n_docs
    r = {"bound": "lds", "kernel": "k_qt_post + k_topk_window (both query chunks)",
         "stage_ms": round(stage_ms, 3), "algorithmic_bytes": alg,
         "achieved": round(alg / (stage_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(alg / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None}
    c = PRUNE_COUNTERS.get(workload)
    if c and _sources_sha1(PRUNE_SOURCES) == PRUNE_SOURCES_SHA1:
        r["traffic"] = c["bytes"]
        r["counted_hbm_gbs"] = round(c["bytes"] / (stage_ms * 1e-3) / 1e9, 1)
        r["counted_hbm_frac"] = round(r["counted_hbm_gbs"] / HBM_PEAK_GBS, 4)
        for key in ("lds_busy", "lds_bank_conflict", "valu_issue", "l2_hit"):
            r[key] = c[key]
    return r


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import gen
    if name == "batched":
        return gen.make("batched"), 1000, 20, ("text-shaped ground space V=100000 d=300 (L2-normalised 200-cluster "
                                               "mixture); 1000000 docs and 4096 queries, sizes 5..500 with "
                                               "P(m)~m^-1.1, Zipf(1.1) words; Quadtree prune to 1000 over all docs, "
                                               "batched Flowtree rerank to top-20")
    if name == "batched_v1m":
        return gen.make("batched", V=1_000_000), 1000, 20, (
            "batched with V=1000000 ground points in R^300 (1.2 GB of coordinates, past the 256 MB "
            "Infinity Cache); 1000000 docs and 4096 queries, sizes 5..500 with P(m)~m^-1.1, Zipf(1.1) "
            "words; Quadtree prune to 1000 over all docs, batched Flowtree rerank to top-20")
    if name == "exhaustive":
        return gen.make("batched", n_queries=64), 0, 20, (
            "exhaustive: the batched ground space and 1000000 docs (V=100000 d=300, sizes 5..500 with "
            "P(m)~m^-1.1, Zipf(1.1) words); 64 queries of the same law, batched Flowtree against every doc "
            "(64M pairs), top-20")
    if name == "text":
        return gen.make("text"), 1000, 20, ("text-shaped: V=100000 d=300, 100000 docs and 1000 queries of 20..200 "
                                            "words; Quadtree prune to 1000, batched Flowtree rerank to top-20")
    if name == "image":
        return gen.make("image"), 0, 10, ("image-shaped: 28x28 grid in R^2, 60000 stroke images and 1000 queries "
                                          "of 100..200 pixels (Q=16); batched Flowtree against all docs, top-10")
    if name == "tiny":
        return gen.make("tiny"), 0, 5, ("tiny: V=2000 points in R^16 (20-component Gaussian mixture), 500 docs and "
                                        "10 queries of 10..30 points; batched Flowtree against all docs, top-5")
    raise SystemExit("unknown workload " + name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0)
    ap.add_argument("--reps", type=int, default=100)
    ap.add_argument("--act-cand", type=int, default=0)
    ap.add_argument("--act-iters", type=int, default=1)
    ap.add_argument("--sk-iters", type=int, default=1)
    ap.add_argument("--trees", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched Flowtree on the default schedule (chunk 4, full occupancy) instead of timing "
                         "ten schedules on the first call; for short profiled runs")
    args = ap.parse_args()
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.workload == "random_model":
        return random_model_experiment(args)
    if args.workload == "recall":
        return recall_experiment(args)
    if args.workload == "grad":
        return grad_bench(args)
    if args.workload in ("act", "sinkhorn", "exact"):
        return rerank_stage(args, args.workload)
    if args.workload == "pipeline":
        return pipeline_bench(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    ds, prune, k, desc = workload(args.workload)
    log("generated %s in %.1fs: V=%d d=%d docs=%d queries=%d nnz=%d" % (
        args.workload, time.time() - t0, ds.V, ds.d, ds.n_docs, ds.n_queries, len(ds.doc_id)))

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    t0 = time.time()
    ix = ft.build_tree(T(ds.X), ds.shift, ds.B, T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass), ds.Q)
    torch.cuda.synchronize()
    info = ix.info()
    log("built index in %.1fs: %s" % (time.time() - t0, info))
    if args.no_autotune:
        ix.set_autotune(0)
    qo, qi, qm = T(ds.q_off), T(ds.q_id), T(ds.q_mass)
    n_q = ds.n_queries

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    stage_qt, stage_ft, kernel_ms, sel_exact = [], [], [], []

    def step():
        """One pass of the whole path: with a prune, the one-call pipeline
        (queries prepared once, flags read once); without, the batched
        Flowtree over all docs."""
        if prune:
            return ft.knn_pipeline(ix, qo, qi, qm, prune, k)
        ev[1].record()
        out = ft.flowtree_knn(ix, qo, qi, qm, k, mode=ft.FT_BATCHED)
        ev[2].record()
        return out

    def two_calls():
        """The same path as two calls (prune, then rerank the candidates)."""
        ev[0].record()
        _, cand = ft.quadtree_knn(ix, qo, qi, qm, prune)
        ev[1].record()
        costs, docs = ft.flowtree_knn(ix, qo, qi, qm, k, cand=cand, mode=ft.FT_BATCHED)
        ev[2].record()
        return cand, costs, docs

    log("warmup x%d (the first call tunes the batched schedule)" % args.warmup)
    for _ in range(max(1, args.warmup)):
        costs, docs = step()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        costs, docs = step()
        torch.cuda.synchronize()
        if prune:
            qt_ms, ft_ms = ix.last_pipeline_stats()
        else:
            qt_ms, ft_ms = 0.0, ev[1].elapsed_time(ev[2])
        stage_qt.append(qt_ms)
        stage_ft.append(ft_ms)
        kernel_ms.append(ix.last_batched_stats()[0])
        sel_exact.append(ix.last_select_exact_rows() if prune else 0)
        log("  step %d: quadtree %.1f ms, flowtree %.1f ms (persistent kernels %.1f ms)" % (
            i, stage_qt[-1], stage_ft[-1], kernel_ms[-1]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    cand = None
    two_call = None
    if prune:
        # the same steps as two calls: the candidates for the byte count and
        # the plain schedule, and the step time the one-call pipeline saves
        cand, c2, d2 = two_calls()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for i in range(args.steps):
            cand, c2, d2 = two_calls()
            torch.cuda.synchronize()
        two_ms = 1000.0 * (time.perf_counter() - t2) / args.steps
        same = bool(torch.equal(d2, docs) and torch.equal(c2.view(torch.int32), costs.view(torch.int32)))
        two_call = {"ms_per_step": round(two_ms, 3), "pipeline_ms_per_step": round(ms_step, 3),
                    "identical_output": same}
        log("two calls: %.1f ms per step vs one-call pipeline %.1f ms (identical output: %s)" % (
            two_ms, ms_step, same))
    n_cols = prune if prune else ds.n_docs
    ft_pairs = n_q * n_cols
    value = ft_pairs / (elapsed / args.steps)
    schedule = ix.last_batched_stats()[1]

    # algorithmic bytes of the Flowtree stage: every candidate doc's items
    # (rank + mass, 8 B) and coordinate rows (4 d B); each query once
    sizes = np.diff(ds.doc_off)
    row_bytes = 8 + 4 * ds.d
    if cand is not None:
        doc_bytes = float(sizes[cand.cpu().numpy()].sum()) * row_bytes
    else:
        doc_bytes = float(n_q) * float(sizes.sum()) * row_bytes
    q_bytes = float(np.diff(ds.q_off).sum()) * row_bytes
    alg_bytes = doc_bytes + q_bytes
    kms = float(np.mean(kernel_ms))
    achieved = alg_bytes / (kms * 1e-3) / 1e9

    plain = None
    if not args.no_plain:
        log("plain one-launch-per-query Flowtree stage on the same candidates")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ft.flowtree_knn(ix, qo, qi, qm, k, cand=cand, mode=ft.FT_PLAIN)
        torch.cuda.synchronize()
        reps = 2
        e0.record()
        for _ in range(reps):
            pc, pd = ft.flowtree_knn(ix, qo, qi, qm, k, cand=cand, mode=ft.FT_PLAIN)
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / reps
        same = bool(torch.equal(pd, docs) and torch.equal(pc, costs))
        plain = {"flowtree_stage_ms": round(pms, 3), "pairs_per_s": round(ft_pairs / (pms * 1e-3), 1),
                 "batched_stage_ms": round(float(np.mean(stage_ft)), 3),
                 "batched_over_plain": round(pms / float(np.mean(stage_ft)), 3),
                 "identical_output": same}
        log("plain: %.1f ms vs batched %.1f ms" % (pms, float(np.mean(stage_ft))))

    copy_gbs = measure_copy_gbs()
    log("device copy: %.0f GB/s" % copy_gbs)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ds, prune, k, n_cols)

    out = {
        "metric": "Flowtree (query,doc) pairs/sec on 1 MI355X, batched vs plain; % HBM roofline",
        "value": round(value, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "queries": n_q, "docs": ds.n_docs, "V": ds.V, "d": ds.d,
                   "prune_k": prune, "k": k, "flowtree_pairs_per_step": ft_pairs},
        "roofline": roofline_block(achieved, kms, alg_bytes, measured_traffic(args.workload), copy_gbs,
                                   "k_flow_persistent (all size classes, one graph)"),
        "roofline_prune": prune_roofline(args.workload, float(np.mean(stage_qt)), n_q, ds.n_docs) if prune else None,
        "stages": {"quadtree_prune_ms": round(float(np.mean(stage_qt)), 3),
                   "prune_select_exact_rows": int(np.max(sel_exact)) if sel_exact else 0,
                   "quadtree_pairs_per_s": round(n_q * ds.n_docs / (float(np.mean(stage_qt)) * 1e-3), 1)
                   if prune else None,
                   "flowtree_batched_ms": round(float(np.mean(stage_ft)), 3),
                   "flowtree_batched_pairs_per_s": round(ft_pairs / (float(np.mean(stage_ft)) * 1e-3), 1),
                   "schedule": schedule},
        "two_calls": two_call,
        "plain": plain,
        "cpu_baseline": cpu,
        "index": info,
    }
    print(json.dumps(out), flush=True)


def measure_copy_gbs(nbytes=1 << 31, reps=5):
    """Read + write rate of a plain device-to-device copy of nbytes (best of
    reps), the measured counterpart of the 8 TB/s HBM figure."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def roofline_block(achieved, kernel_ms, alg_bytes, traffic, copy_gbs, kernel):
    """The roofline object of the bench line: algorithmic bytes per launch
    over the kernel's live duration against the HBM peak, with the counted
    HBM bytes (rocprofv3 FETCH_SIZE / WRITE_SIZE, when taken on these
    sources) as a rate and a fraction of peak beside it, and the measured
    copy rate."""
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "kernel_ms": round(kernel_ms, 3), "algorithmic_bytes": alg_bytes,
         "copy_measured_gbs": round(copy_gbs, 1)}
    if traffic:
        counted = traffic / (kernel_ms * 1e-3) / 1e9
        r["counted_hbm_gbs"] = round(counted, 1)
        r["counted_hbm_frac"] = round(counted / HBM_PEAK_GBS, 4)
    return r


RANDOM_MODEL_SETTINGS = (
    # (d, s, eps, N values): the two settings of the paper's random-data figure
    (10, 10, 0.25, (100, 200, 500, 1000, 2000, 5000, 10000)),
    (10, 100, 0.4, (200, 500, 1000, 2000)),
)


def random_model_experiment(args):
    """Section 3.2 / 4.1: N points uniform on the sphere, a planted doc of s
    of them, a query of s points each within eps of its planted point.  The
    competitors are the planted doc's single-swap neighbours (one x_k
    replaced by any other of the N points, s * (N - s) docs: the failure
    event of the analysis is such a swap).  A repetition succeeds for an
    estimate when the planted doc is strictly the nearest of all; one index
    and one query per repetition.  Also reported: how often the planted
    pair's Flowtree value equals the planted matching's cost (the tree flow
    is then optimal, which the analysis shows for an event independent of
    N)."""
    if args.gpus != 1:
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    results = []
    pairs = 0
    gpu_s = 0.0
    t_all = time.time()
    for d, s, eps, Ns in RANDOM_MODEL_SETTINGS:
        for N in Ns:
            rng = np.random.default_rng(1000003 * N + 97 * s + d)
            ok_qt = ok_ft = exact = 0
            rnd_qt = rnd_ft = 0.0     # success with ties at the minimum broken uniformly at random
            tie_qt = tie_ft = 0       # planted doc at the minimum together with another doc
            zero = torch.zeros(1, dtype=torch.int64, device=dev)
            planted_cost = torch.empty(1, dtype=torch.float32, device=dev)
            for rep in range(args.reps):
                if rep and rep % 25 == 0:
                    log("  N=%d s=%d: %d of %d repetitions" % (N, s, rep, args.reps))
                ds = gen.random_model_swaps(rng, N, d, s, eps)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Xd = T(ds.X)
                ix = ft.build_tree(Xd, ds.shift, ds.B, T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass), ds.Q)
                q = (T(ds.q_off), T(ds.q_id), T(ds.q_mass))
                keys, kd = ft.quadtree_knn(ix, *q, 2)
                costs, fd = ft.flowtree_knn(ix, *q, 2, mode=ft.FT_PLAIN)
                torch.cuda.synchronize()
                gpu_s += time.perf_counter() - t0
                # the planted pair alone: is its Flowtree value the planted
                # matching's cost (the tree flow optimal, as under the event
                # of the analysis)?
                ft.flowtree_cost_grad(ix, Xd, *q, zero, zero, ft.FT_FWD, cost=planted_cost)
                x, y = ds.X[ds.extra["planted"]].astype(np.float64), ds.X[ds.q_id].astype(np.float64)
                match = float(np.mean(np.linalg.norm(x - y, axis=1)))
                exact += int(abs(float(planted_cost.cpu()[0]) - match) <= 1e-5 * match)
                keys = keys.cpu().numpy().view(np.uint64)[0]
                costs, kd, fd = costs.cpu().numpy()[0], kd.cpu().numpy()[0], fd.cpu().numpy()[0]
                ok_qt += int(kd[0] == 0 and keys[0] < keys[1])
                ok_ft += int(fd[0] == 0 and costs[0] < costs[1])
                # every doc's value, for the tie rules: how many docs share
                # the smallest value with the planted one
                pq = torch.zeros(ds.n_docs, dtype=torch.int64, device=dev)
                pd = torch.arange(ds.n_docs, dtype=torch.int64, device=dev)
                allk = ft.quadtree_pairs(ix, *q, pq, pd).cpu().numpy().view(np.uint64)
                allc = torch.empty(ds.n_docs, dtype=torch.float32, device=dev)
                ft.flowtree_cost_grad(ix, Xd, *q, pq, pd, ft.FT_FWD, cost=allc)
                allc = allc.cpu().numpy()
                for vals, name in ((allk, "qt"), (allc, "ft")):
                    at_min = vals == vals.min()
                    if at_min[0]:
                        share = 1.0 / at_min.sum()
                        if name == "qt":
                            rnd_qt += share
                            tie_qt += int(at_min.sum() > 1)
                        else:
                            rnd_ft += share
                            tie_ft += int(at_min.sum() > 1)
                pairs += 2 * ds.n_docs
                del ix
            R = args.reps
            results.append({"d": d, "s": s, "eps": eps, "N": N, "docs": 1 + s * (N - s), "reps": R,
                             "quadtree_success": ok_qt / R, "flowtree_success": ok_ft / R,
                             "quadtree_success_random_ties": round(rnd_qt / R, 4),
                             "flowtree_success_random_ties": round(rnd_ft / R, 4),
                             "quadtree_tied_at_min": tie_qt / R, "flowtree_tied_at_min": tie_ft / R,
                             "flowtree_planted_exact": exact / R})
            log("random model d=%d s=%d eps=%.2f N=%d: strict quadtree %.2f flowtree %.2f; random ties "
                "quadtree %.3f flowtree %.3f; tied at min quadtree %.2f flowtree %.2f (planted exact %.2f)" % (
                    d, s, eps, N, ok_qt / R, ok_ft / R, rnd_qt / R, rnd_ft / R, tie_qt / R, tie_ft / R, exact / R))
    out = {"metric": "random-model planted nearest neighbour recovered (fraction of repetitions), "
                     "Quadtree vs Flowtree, as N grows",
           "unit": "fraction", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "random model of Section 3.2: N uniform points on S^(d-1), planted doc of s "
                                  "points, query within eps of it; competitors = single-swap docs"},
           "results": results,
           "gpu_seconds": round(gpu_s, 2), "wall_seconds": round(time.time() - t_all, 2),
           "pairs_per_s_incl_index_build": round(pairs / gpu_s, 1)}
    print(json.dumps(out), flush=True)


def grad_bench(args):
    """Differentiation workload: V = 50k points in R^300 (text law), 256
    (query, doc) pairs with supports 20..200.  One step = the forward pass
    (Flowtree cost of every pair; saves the flows) and the backward pass
    (gradients of sum_p g_p cost_p w.r.t. X and both weight vectors, tree and
    flow pattern frozen), gradient buffers cleared in the step.  value =
    pairs / step time.  roofline: algorithmic bytes (items and coordinate
    rows read by each pass, plus one fp32 gradient row per item written) over
    the device time of the two passes."""
    if args.gpus != 1:
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    ds = gen.make("grad")
    ix = ft.build_tree(T(ds.X), ds.shift, ds.B, T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass), ds.Q)
    X = T(ds.X)
    q = (T(ds.q_off), T(ds.q_id), T(ds.q_mass))
    pq, pd = T(ds.extra["pair_q"]), T(ds.extra["pair_d"])
    n_p = len(ds.extra["pair_q"])
    cost = torch.empty(n_p, dtype=torch.float32, device=dev)
    g = torch.linspace(0.5, 1.5, n_p, dtype=torch.float32, device=dev)
    gX = torch.zeros_like(X)
    gq = torch.zeros(len(ds.q_id), dtype=torch.float32, device=dev)
    gd = torch.zeros(len(ds.doc_id), dtype=torch.float32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step():
        ev[0].record()
        ft.flowtree_cost_grad(ix, X, *q, pq, pd, ft.FT_FWD, cost=cost)
        ev[1].record()
        gX.zero_()
        gq.zero_()
        gd.zero_()
        ft.flowtree_cost_grad(ix, X, *q, pq, pd, ft.FT_BWD, grad_out=g, grad_X=gX, grad_qmass=gq, grad_dmass=gd)
        ev[2].record()

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    fwd, bwd = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        fwd.append(ev[0].elapsed_time(ev[1]))
        bwd.append(ev[1].elapsed_time(ev[2]))
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    sq = np.diff(ds.q_off)[ds.extra["pair_q"]]
    sdd = np.diff(ds.doc_off)[ds.extra["pair_d"]]
    items = float((sq + sdd).sum())
    row = 4.0 * ds.d
    alg = 2.0 * items * (8.0 + row) + items * row
    dev_ms = float(np.mean(fwd) + np.mean(bwd))
    achieved = alg / (dev_ms * 1e-3) / 1e9
    log("grad: forward %.3f ms, backward %.3f ms (events), step %.3f ms" % (np.mean(fwd), np.mean(bwd), ms_step))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        Tr = oracle.Tree(ds.X, ds.shift, ds.B)
        done = 0
        t0 = time.perf_counter()
        for p in range(n_p):
            qq, dd = ds.extra["pair_q"][p], ds.extra["pair_d"][p]
            a, b = ds.doc_off[dd], ds.doc_off[dd + 1]
            qa, qb = ds.q_off[qq], ds.q_off[qq + 1]
            _, fl = Tr.flowtree(ds.doc_id[a:b], ds.doc_mass[a:b], ds.q_id[qa:qb], ds.q_mass[qa:qb], Q=ds.Q)
            oracle.frozen_grad(ds.X, ds.doc_id[a:b], ds.q_id[qa:qb], fl, ds.doc_mass[a:b] / 2.0 ** ds.Q,
                               ds.q_mass[qa:qb] / 2.0 ** ds.Q)
            done += 1
            if time.perf_counter() - t0 > 15.0:
                break
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 2), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": "%d of %d pairs: oracle Flowtree (C) then the float64 frozen cost gradient (numpy), "
                         "single-threaded" % (done, n_p)}
    out = {"metric": "Flowtree cost forward + backward (query, doc) pairs/sec on 1 MI355X",
           "value": round(n_p / (elapsed / args.steps), 1), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "differentiation: V=50000 points in R^300 (L2-normalised 200-cluster mixture), "
                                  "256 (query, doc) pairs with supports 20..200; gradient of sum_p g_p cost_p "
                                  "w.r.t. X and both weight vectors, tree and flow frozen",
                      "pairs": n_p, "V": ds.V, "d": ds.d},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "k_flow_save + k_flow_bwd (forward and backward passes)",
                        "kernel_ms": round(dev_ms, 4), "algorithmic_bytes": alg},
           "stages": {"forward_ms": round(float(np.mean(fwd)), 4), "backward_ms": round(float(np.mean(bwd)), 4)},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


RECALL_AT = (1, 2, 4, 8, 16, 32, 64, 128)


def recall_experiment(args):
    """Accuracy of the estimates as nearest-neighbour rankers (Section 4.2:
    recall@m = the fraction of queries whose true nearest neighbour, by exact
    W1, is among the top m candidates of a method; the randomised tree methods
    reported as mean and standard deviation over independent random shifts,
    five in the paper).  Three synthetic worlds stand in for the paper's
    datasets: the tiny-config law (R^16 mixture, 10..30 points), the text law
    (R^300, 20..200 words) and stroke images on the 28x28 grid.  Every value
    comes from the GPU path: exact W1 over all docs gives the truth; Quadtree,
    the eps-weighted Quadtree (eps = 1 / log2 of the mean support, the
    weighting of the uniform-distribution Flowtree bound) and Flowtree rank all
    docs under each shift; R-WMD, ACT-1 and Sinkhorn-1 (deterministic) once."""
    if args.gpus != 1:
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    worlds = [
        ("tiny configuration: V=2000 in R^16, 20-cluster mixture; 500 docs, 10 queries of 10..30 points",
         gen.make("tiny")),
        ("tiny law: V=2000 in R^16, 20-cluster mixture; 1000 docs, 200 queries of 10..30 points",
         gen.make("tiny", n_docs=1000, n_queries=200)),
        ("text law: V=20000 in R^300, L2-normalised 200-cluster mixture; 1000 docs, 50 queries of 20..200 words",
         gen.make("text", V=20000, n_docs=1000, n_queries=50)),
        ("image law: 28x28 grid; 1000 stroke images, 50 queries of 100..200 pixels (Q=16)",
         gen.make("image", n_docs=1000, n_queries=50)),
    ]
    M = max(RECALL_AT)
    t_all = time.time()
    results = []
    for desc, ds in worlds:
        n_q, n_d = ds.n_queries, ds.n_docs
        docs = (T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass))
        q = (T(ds.q_off), T(ds.q_id), T(ds.q_mass))
        Xd = T(ds.X)
        ix = ft.build_tree(Xd, ds.shift, ds.B, *docs, ds.Q)
        t0 = time.perf_counter()
        _, truth = ft.exact_knn(ix, *q, 1)
        torch.cuda.synchronize()
        exact_s = time.perf_counter() - t0
        truth = truth.cpu().numpy()[:, 0]
        log("%s: exact W1 of %d pairs in %.1fs" % (desc, n_q * n_d, exact_s))

        def recall(ranked):
            ranked = np.asarray(ranked)
            hit = ranked == truth[:, None]
            first = np.where(hit.any(axis=1), hit.argmax(axis=1), M)
            return [round(float(np.mean(first < m)), 4) for m in RECALL_AT]

        mean_s = float(np.mean(np.diff(ds.q_off)))
        eps = 1.0 / np.log2(mean_s)
        cand_all = T(np.tile(np.arange(n_d, dtype=np.int64), (n_q, 1)))
        per = {"quadtree": [], "quadtree_eps": [], "flowtree": []}
        rng = np.random.default_rng(1234)
        for tree in range(args.trees):
            shift = gen.random_shift(rng, ds.d, ds.B)
            tix = ft.build_tree(Xd, shift, ds.B, *docs, ds.Q)
            _, qd = ft.quadtree_knn(tix, *q, M)
            _, qe = ft.quadtree_eps_knn(tix, *q, M, cand_all, eps)
            _, fd = ft.flowtree_knn(tix, *q, M, mode=ft.FT_BATCHED)
            per["quadtree"].append(recall(qd.cpu().numpy()))
            per["quadtree_eps"].append(recall(qe.cpu().numpy()))
            per["flowtree"].append(recall(fd.cpu().numpy()))
            del tix
        row = {"world": desc, "docs": n_d, "queries": n_q, "trees": args.trees, "eps": round(eps, 4),
               "recall_at": list(RECALL_AT), "exact_w1_seconds": round(exact_s, 2)}
        for name, v in per.items():
            v = np.asarray(v)
            row[name] = {"mean": [round(float(x), 4) for x in v.mean(axis=0)],
                         "std": [round(float(x), 4) for x in v.std(axis=0)]}
        for name, f in (("rwmd", lambda: ft.act_knn(ix, *q, M, iters=0)),
                        ("act1", lambda: ft.act_knn(ix, *q, M, iters=1)),
                        ("sinkhorn1", lambda: ft.sinkhorn_knn(ix, *q, M, iters=1))):
            _, dd = f()
            row[name] = recall(dd.cpu().numpy())
        log("  recall@%s" % (list(RECALL_AT),))
        for name in ("quadtree", "quadtree_eps", "flowtree"):
            log("  %-13s %s +- %s" % (name, row[name]["mean"], row[name]["std"]))
        for name in ("rwmd", "act1", "sinkhorn1"):
            log("  %-13s %s" % (name, row[name]))
        results.append(row)
        del ix
    out = {"metric": "recall@m of the true (exact W1) nearest neighbour, per method",
           "unit": "fraction", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "accuracy experiment of Section 4.2 on synthetic stand-ins; tree methods over "
                                  "%d random shifts" % args.trees},
           "results": results, "wall_seconds": round(time.time() - t_all, 2)}
    print(json.dumps(out), flush=True)


FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense fp64 matrix peak


def rerank_stage(args, method):
    """A quadratic-time stage the paper's pipelines put after Flowtree
    (Section 4.3): on the batched workload, Quadtree prunes every doc to
    1000, batched Flowtree keeps the best C of those, and ACT-I (method
    "act") or Sinkhorn-I ("sinkhorn") ranks the C to the top-20.  One step is
    that call for all 4096 queries; the Quadtree and Flowtree stages run
    beforehand and are timed beside it (second calls).  value = pairs per
    second of the call (query preparation and select included); roofline:
    the inner-product contraction of the stage's kernels (2 s_q s_d d flops
    per pair, unpadded; fp64 on the matrix cores) against the fp64 matrix
    peak, over their device time."""
    if args.gpus != 1:
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    C = args.act_cand or (20 if method == "exact" else 100)
    k = 5 if method == "exact" else 20
    iters = args.act_iters if method == "act" else args.sk_iters
    name = {"act": "ACT-%d" % iters, "sinkhorn": "Sinkhorn-%d" % iters, "exact": "exact W1"}[method]

    def call():
        if method == "act":
            return ft.act_knn(ix, *q, k, iters=iters, cand=fdocs)
        if method == "sinkhorn":
            return ft.sinkhorn_knn(ix, *q, k, iters=iters, cand=fdocs)
        return ft.exact_knn(ix, *q, k, cand=fdocs)
    t0 = time.time()
    ds, prune, _, desc = workload("batched")
    log("generated batched workload in %.1fs" % (time.time() - t0))

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    ix = ft.build_tree(T(ds.X), ds.shift, ds.B, T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass), ds.Q)
    q = (T(ds.q_off), T(ds.q_id), T(ds.q_mass))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    _, cand = ft.quadtree_knn(ix, *q, prune)
    _, fdocs = ft.flowtree_knn(ix, *q, C, cand=cand, mode=ft.FT_BATCHED)
    ev[0].record()
    _, cand = ft.quadtree_knn(ix, *q, prune)
    ev[1].record()
    _, fdocs = ft.flowtree_knn(ix, *q, C, cand=cand, mode=ft.FT_BATCHED)
    ev[2].record()
    torch.cuda.synchronize()
    qt_ms, ft_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    log("quadtree %.1f ms, flowtree %.1f ms" % (qt_ms, ft_ms))
    n_q = ds.n_queries
    log("warmup x%d" % args.warmup)
    for _ in range(max(1, args.warmup)):
        costs, docs = call()
    torch.cuda.synchronize()
    kms = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        costs, docs = call()
        kms.append(ix.last_rerank_ms())
        log("  step %d: %s kernels %.2f ms" % (i, name, kms[-1]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    pairs = n_q * C
    fd = fdocs.cpu().numpy()
    sq = np.diff(ds.q_off)
    sd = np.diff(ds.doc_off)[fd]
    flops = float(2.0 * ds.d * (sq[:, None].astype(np.float64) * sd).sum())
    kmean = float(np.mean(kms))
    achieved = flops / (kmean * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        cpu = rerank_cpu_baseline(ds, fd, method, iters)
    out = {
        "metric": "%s (query, candidate) pairs/sec on 1 MI355X (the stage after Flowtree)" % name,
        "value": round(pairs / (elapsed / args.steps), 1), "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc + "; then batched Flowtree keeps the best %d candidates and %s ranks them "
                                      "to the top-%d" % (C, name, k),
                   "queries": n_q, "candidates": C, "iters": iters, "k": k, "act_pairs_per_step": pairs},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": {"act": "k_act (all query classes)", "sinkhorn": "k_sinkhorn",
                                "exact": "k_exact"}[method],
                     "kernel_ms": round(kmean, 3),
                     "algorithmic_flops": flops},
        "stages": {"quadtree_prune_ms": round(qt_ms, 3), "flowtree_batched_ms": round(ft_ms, 3),
                   "rerank_call_ms": round(ms_step, 3), "rerank_kernels_ms": round(kmean, 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def pipeline_bench(args):
    """The paper's prefetch-and-prune pipeline (Section 4.3) end to end on
    the batched workload: Quadtree prunes every doc to 1000, batched
    Flowtree keeps 100, ACT-1 keeps 5, exact W1 ranks those 5 and keeps the
    best.  One step is the four calls for all 4096 queries; value = queries
    per second through all four.  Each stage's time comes from events
    between the calls."""
    if args.gpus != 1:
        print("bench.py measures one GPU only", file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_1910_04126_amd as ft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    C = (1000, 100, 5, 1)
    t0 = time.time()
    ds = gen.make("batched")
    desc = ("text-shaped ground space V=100000 d=300 (L2-normalised 200-cluster mixture); 1000000 docs and 4096 "
            "queries, sizes 5..500 with P(m)~m^-1.1, Zipf(1.1) words; Quadtree prunes every doc to 1000, batched "
            "Flowtree keeps 100, ACT-1 keeps 5, exact W1 ranks those to the top-1")
    log("generated batched workload in %.1fs" % (time.time() - t0))

    def T(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    ix = ft.build_tree(T(ds.X), ds.shift, ds.B, T(ds.doc_off), T(ds.doc_id), T(ds.doc_mass), ds.Q)
    if args.no_autotune:
        ix.set_autotune(0)
    q = (T(ds.q_off), T(ds.q_id), T(ds.q_mass))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step():
        ev[0].record()
        _, fdocs = ft.knn_pipeline(ix, *q, C[0], C[1])
        ev[1].record()
        _, adocs = ft.act_knn(ix, *q, C[2], iters=1, cand=fdocs)
        ev[2].record()
        w, best = ft.exact_knn(ix, *q, C[3], cand=adocs)
        ev[3].record()
        return w, best

    log("warmup x%d" % args.warmup)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    st = {"quadtree_flowtree": [], "act": [], "exact": []}
    t_start = time.perf_counter()
    for i in range(args.steps):
        w, best = step()
        torch.cuda.synchronize()
        st["quadtree_flowtree"].append(ev[0].elapsed_time(ev[1]))
        st["act"].append(ev[1].elapsed_time(ev[2]))
        st["exact"].append(ev[2].elapsed_time(ev[3]))
        log("  step %d: Quadtree+Flowtree %.1f ms, ACT-1 %.1f ms, exact W1 %.1f ms" % (
            i, st["quadtree_flowtree"][-1], st["act"][-1], st["exact"][-1]))
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    n_q = ds.n_queries
    cpu = None if args.no_cpu_baseline else pipeline_cpu_baseline(ds, C)
    out = {
        "metric": "queries/sec through the four-stage pipeline (Quadtree, Flowtree, ACT-1, exact W1) on 1 MI355X",
        "value": round(n_q / (elapsed / args.steps), 2), "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "queries": n_q, "candidates": list(C)},
        "roofline": None,
        "stages": {k: round(float(np.mean(v)), 3) for k, v in st.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def pipeline_cpu_baseline(ds, C):
    """The oracle through the same four stages (Quadtree on every doc, top
    C[0]; Flowtree, top C[1]; ACT-1 in float64, top C[2]; exact W1 by LP,
    top C[3]) for whole queries in order, one thread, for about 20 s."""
    import oracle
    Tr = oracle.Tree(ds.X, ds.shift, ds.B)
    docs = np.arange(ds.n_docs)
    done = 0
    t_start = time.perf_counter()
    for qq in range(ds.n_queries):
        U = Tr.quadtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass,
                              np.full(ds.n_docs, qq), docs, ds.Q)
        _, c1 = oracle.topk(U, docs, C[0])
        F = Tr.flowtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass,
                              np.full(len(c1), qq), c1, ds.Q)
        _, c2 = oracle.topk(F, c1, C[1])
        A = oracle.act_pairs(ds.X, ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass,
                             np.full(len(c2), qq), c2, ds.Q, 1)
        _, c3 = oracle.topk(A, c2, C[2])
        qa, qb = ds.q_off[qq], ds.q_off[qq + 1]
        W = np.array([oracle.exact_w1_lp(ds.X, ds.doc_id[ds.doc_off[d]:ds.doc_off[d + 1]],
                                         ds.doc_mass[ds.doc_off[d]:ds.doc_off[d + 1]],
                                         ds.q_id[qa:qb], ds.q_mass[qa:qb], ds.Q) for d in c3])
        oracle.topk(W, c3, C[3])
        done += 1
        if time.perf_counter() - t_start > 20.0:
            break
    el = time.perf_counter() - t_start
    return {"value": round(done / el, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": "%d of %d queries in order through the four stages (C oracle for Quadtree and "
                      "Flowtree, float64 numpy ACT-1, LP by HiGHS for exact W1), one thread" % (done, ds.n_queries)}


def rerank_cpu_baseline(ds, fdocs, method, iters):
    """The float64 oracle (ACT, Sinkhorn or exact W1) on a bounded sample of the same
    pairs (queries in order, all their candidates), single-threaded."""
    import oracle
    budget = 15.0
    done = 0
    t_start = time.perf_counter()
    for qq in range(ds.n_queries):
        pq, pd = np.full(fdocs.shape[1], qq), fdocs[qq]
        if method == "exact":
            for d in pd:
                a, b = ds.doc_off[d], ds.doc_off[d + 1]
                qa, qb = ds.q_off[qq], ds.q_off[qq + 1]
                oracle.exact_w1_lp(ds.X, ds.doc_id[a:b], ds.doc_mass[a:b], ds.q_id[qa:qb], ds.q_mass[qa:qb], ds.Q)
        else:
            f = oracle.act_pairs if method == "act" else oracle.sinkhorn_pairs
            f(ds.X, ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass, pq, pd, ds.Q, iters)
        done += 1
        if time.perf_counter() - t_start > budget:
            break
    el = time.perf_counter() - t_start
    return {"value": round(done * fdocs.shape[1] / el, 2), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": "%d of %d queries, all %d candidates each, float64 oracle (%s)" %
                      (done, ds.n_queries, fdocs.shape[1], "LP by HiGHS" if method == "exact" else "numpy")}


def calibrate_copy(nbytes):
    """Copy a device buffer of nbytes five times (one copy kernel each), so
    the counters' FETCH_SIZE / WRITE_SIZE per dispatch can be compared with
    the nbytes actually moved."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)


def cpu_threads():
    """Host threads for the all-cores oracle leg: the CPUs this process may
    run on, capped by OMP_NUM_THREADS when it is set (the GPU machine gives a
    one-GPU job 16)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


# With no prune over this many docs, one query of the CPU oracle takes far
# longer than the sample's budget: the sample is then cut into (query, block
# of docs) items, each ranked on its own.
ORACLE_DOC_BLOCK = 2000
ORACLE_BLOCKED_DOCS = 100_000


def _oracle_pipeline(ds, prune, k, n_cols, threads, budget):
    """Whole-pipeline queries of the CPU oracle (Quadtree on every doc,
    top-`prune`, Flowtree on those, top-k; or Flowtree on every doc when
    prune = 0), one query per thread at a time, each thread with its own
    oracle tree, until `budget` seconds have passed.  Without a prune over
    more than ORACLE_BLOCKED_DOCS docs an item is one query against a block
    of ORACLE_DOC_BLOCK docs (Flowtree, top-k of the block).  Returns
    (Flowtree pairs done, seconds, items done)."""
    import itertools
    import threading

    import oracle
    trees = [oracle.Tree(ds.X, ds.shift, ds.B) for _ in range(threads)]
    docs = np.arange(ds.n_docs)
    blocked = not prune and ds.n_docs > ORACLE_BLOCKED_DOCS
    n_blocks = -(-ds.n_docs // ORACLE_DOC_BLOCK) if blocked else 1
    next_item = itertools.count()
    lock = threading.Lock()
    done = [0] * threads
    pairs = [0] * threads
    t_start = time.perf_counter()

    def worker(i):
        Tr = trees[i]
        while time.perf_counter() - t_start < budget:
            with lock:
                item = next(next_item)
            q, b = divmod(item, n_blocks)
            if q >= ds.n_queries:
                return
            if prune:
                U = Tr.quadtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass,
                                      np.full(ds.n_docs, q), docs, ds.Q)
                _, cand = oracle.topk(U, docs, prune)
            elif blocked:
                cand = docs[b * ORACLE_DOC_BLOCK:(b + 1) * ORACLE_DOC_BLOCK]
            else:
                cand = docs
            F = Tr.flowtree_pairs(ds.q_off, ds.q_id, ds.q_mass, ds.doc_off, ds.doc_id, ds.doc_mass,
                                  np.full(len(cand), q), cand, ds.Q)
            oracle.topk(F, cand, min(k, len(cand)))
            done[i] += 1
            pairs[i] += len(cand)

    ths = [threading.Thread(target=worker, args=(i,)) for i in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    return sum(pairs), time.perf_counter() - t_start, sum(done)


def cpu_baseline(ds, prune, k, n_cols):
    """The CPU oracle on a bounded sample of the same workload: the full
    pipeline for whole queries (Quadtree against every doc, top-`prune`,
    Flowtree on those candidates, top-k), once on one thread (as the paper
    times its implementation) and once on all host cores with one query per
    thread; scaled to Flowtree pairs per second of that pipeline.  The main
    value is the all-cores leg."""
    blocked = not prune and ds.n_docs > ORACLE_BLOCKED_DOCS
    what = (("Quadtree on all %d docs, top-%d, Flowtree, top-%d" % (ds.n_docs, prune, k)) if prune else
            ("Flowtree on blocks of %d of the %d docs, top-%d of each block" % (ORACLE_DOC_BLOCK, ds.n_docs, k))
            if blocked else ("Flowtree on all %d docs, top-%d" % (ds.n_docs, k)))
    unit = "(query, doc block) items" if blocked else "queries"
    p1, t1, n1 = _oracle_pipeline(ds, prune, k, n_cols, 1, 15.0)
    log("cpu baseline: 1 thread, %d %s in %.1fs" % (n1, unit, t1))
    nt = cpu_threads()
    pn, tn, nn = _oracle_pipeline(ds, prune, k, n_cols, nt, 15.0)
    log("cpu baseline: %d threads, %d %s in %.1fs" % (nt, nn, unit, tn))
    return {"value": round(pn / tn, 2), "unit": "pairs/s", "cores": nt, "kind": "oracle",
            "sample": "%d %s of the %d queries through the whole pipeline (%s), C oracle on %d host threads, "
                      "one item per thread; pairs/s counts the Flowtree pairs of those items" %
                      (nn, unit, ds.n_queries, what, nt),
            "single_thread": {"value": round(p1 / t1, 2), "unit": "pairs/s", "cores": 1,
                              "sample": "%d %s, same pipeline, one thread" % (n1, unit)}}


if __name__ == "__main__":
    main()
