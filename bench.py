"""Benchmark of the HENN search hot path on one MI355X.

Workload (default): 1,000,000 x 128 Gaussian mixture (100 clusters, sigma
0.3), 10,000 queries from the same mixture, L2, k = 10, kNN graph of degree
32 plus reverse edges (60 slots) per layer.  Build once (timed and reported separately), then sweep the beam
width for the FP32 form and the BF16 / FP8 forms (FP32 re-rank of 4k
candidates), pick for every form the smallest beam width whose Recall@10
reaches 0.95, and time exactly --steps batched searches of the best form.

Prints ONE JSON line (rank 0, N = 1).  Recall is measured against the exact
FP64 k-NN of every query (the oracle's matrix-product route); the same CPU leg
times the oracle's own search on the host cores (the cpu_baseline object).
The default run also measures the adversarial-layout workload (1M x 96 points
on a curve with exponentially shrinking gaps, BF16 rows, FP32 re-rank of 4k)
as an extra key.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GRAM = {"split": 0, "fp32": 1}  # kNN graph Gram tiles (build param gram)
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="gmm100_1M_d128")
    ap.add_argument("--n", type=int, default=None, help="fewer points (smoke runs)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--efs", default="16,24,32,48,64,72,80,84,88,92,96,104,112,128,160,192,256")
    ap.add_argument("--forms", default="f32,bf16,fp8")
    ap.add_argument("--gt-sample", type=int, default=0,
                    help="queries with exact ground truth (0 = all)")
    ap.add_argument("--no-adversarial", action="store_true",
                    help="skip the 1M x 96 adversarial-layout measurement")
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", default="knn_sym")
    ap.add_argument("--sampler", default="draws", choices=["draws", "halving"],
                    help="layer sampler: Alg. 2 draws or Alg. 3 halving")
    ap.add_argument("--ef-construction", type=int, default=256, help="NSW insertion beam")
    ap.add_argument("--insert-shift", type=int, default=3, help="NSW batch = inserted >> shift")
    ap.add_argument("--degree", type=int, default=32)
    ap.add_argument("--max-degree", type=int, default=60)
    ap.add_argument("--gram", default="split", choices=["split", "fp32"],
                    help="kNN graph Gram tiles: split BF16 (default) or FP32 matrix cores")
    ap.add_argument("--root-max", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--shape", default=None,
                    help="fixed launch shape 'lanes,waves,vis_bits,persistent' instead of the "
                         "autotuner (profiling runs use the shape the default run chose)")
    ap.add_argument("--mode", default="search",
                    choices=["search", "batched", "serving", "worstcase", "dynamic"],
                    help="search: the metric's ef sweep and timed steps; batched: one hipGraph "
                         "of a mixed-k / mixed-ef persistent batch (10M x 128, FP8 by default); "
                         "worstcase: eps-net against random layers on skewed data; dynamic: "
                         "Insert / Delete on an NSW index")
    ap.add_argument("--wc-runs", type=int, default=8, help="worstcase: builds per configuration")
    ap.add_argument("--wc-rho-runs", type=int, default=100,
                    help="worstcase: runs per recall-bound configuration")
    ap.add_argument("--wc-rho-nq", type=int, default=200,
                    help="worstcase: queries per recall-bound run")
    ap.add_argument("--wc-parts", default="hops,rho",
                    help="worstcase: hops (hop and query-time study), rho (recall bound)")
    ap.add_argument("--wc-nq", type=int, default=1000, help="worstcase: queries per configuration")
    ap.add_argument("--wc-c0d", type=float, default=0.32,
                    help="worstcase: c0 * d of Eq. (1) for the eps-net layers")
    ap.add_argument("--wc-lam", type=float, default=32.0, help="worstcase: skew of the n / d sweeps")
    ap.add_argument("--storage", default="fp8", help="batched mode storage form")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100000,
                    help="requests of the serving runs (cycling through the queries)")
    ap.add_argument("--serve-slots", type=int, default=8192)
    ap.add_argument("--serve-pool-mb", type=int, default=128)
    ap.add_argument("--serve-steps", type=int, default=128)
    ap.add_argument("--serve-root-max", type=int, default=0,
                    help="serving mode: complete-root size limit (0 = greedy root)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def _cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with its family / model /
    stepping numbers (a virtualised host may give only a short name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first processor's block
                k, _, v = line.partition(":")
                info[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    name = info.get("model name", "unknown")
    nums = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    return f"{name} ({', '.join(nums)})" if nums else name


def cpu_threads():
    """Threads of the CPU legs: the process's affinity mask, at most 16 (the
    host's CPU share per GPU).  Returns (threads, affinity size, nproc)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return max(1, min(aff, 16)), aff, os.cpu_count() or aff


def quality(ids, dist, gt_dist, X, Q, sample, metric):
    """Per-query tie-tolerant Recall@k on the sampled queries (a returned id
    counts when its FP64 distance is at most the true k-th; the sums run in a
    different order than the oracle's, so 1e-9 relative is allowed), and the
    returned distances' error against FP64 recomputation: max / mean relative
    error and, per query, the sum of the returned FP64 distances over the sum
    of the true ones (L2; 1 = exact), averaged over the queries (a ratio of
    sums, so that near-zero true distances do not dominate)."""
    k = gt_dist.shape[1]
    I = ids[sample][:, :k]
    ok = I >= 0
    xs = X[np.maximum(I, 0)].astype(np.float64)
    qv = Q[sample].astype(np.float64)[:, None, :]
    dd = ((xs - qv) ** 2).sum(-1) if metric == 0 else -(xs * qv).sum(-1)
    kth = gt_dist[:, k - 1][:, None]
    hit = ok & (dd <= kth + 1e-9 * np.abs(kth))
    per_q = hit.sum(1) / float(k)
    rec = float(per_q.mean())
    ci = float(1.96 * per_q.std(ddof=1) / np.sqrt(len(per_q))) if len(per_q) > 1 else None
    dsel = dist[sample][:, :k].astype(np.float64)
    err = np.abs(dsel - dd)[ok] / np.maximum(np.abs(dd[ok]), 1e-30)
    ratio = None
    if metric == 0:
        got_sum = np.where(ok, dd, 0.0).sum(1)
        true_sum = np.where(ok, gt_dist, 0.0).sum(1)
        ratio = got_sum / np.maximum(true_sum, 1e-30)
    return {"recall": rec, "recall_ci95": ci,
            "max_rel_err": float(err.max()) if err.size else 0.0,
            "mean_rel_err": float(err.mean()) if err.size else 0.0,
            "mean_dist_ratio": float(ratio.mean()) if ratio is not None and ratio.size else None}


def exact_knn(X, Q, k, metric=0):
    """Ground truth of the measurements: the exact k nearest neighbours of
    each query by brute force in FP64 with plain torch on the GPU (L2:
    squared distance, IP: negated inner product), then the kept distances
    recomputed directly in FP64 on the host.  Returns host arrays (ids int64,
    distances float64), rows sorted by distance."""
    import torch
    dev = torch.device("cuda:0")
    X64 = torch.from_numpy(np.ascontiguousarray(X)).to(dev, torch.float64)
    xn = (X64 * X64).sum(1)
    n = X.shape[0]
    chunk = int(max(1, min(256, (1 << 31) // max(n, 1))))
    ids = np.empty((Q.shape[0], k), np.int64)
    for s in range(0, Q.shape[0], chunk):
        q = torch.from_numpy(np.ascontiguousarray(Q[s:s + chunk])).to(dev, torch.float64)
        g = q @ X64.T
        dd = xn[None, :] - 2.0 * g + (q * q).sum(1)[:, None] if metric == 0 else -g
        ids[s:s + chunk] = torch.topk(dd, k, dim=1, largest=False, sorted=True)[1].cpu().numpy()
        del g, dd
    del X64, xn
    xs = X[ids].astype(np.float64)
    qv = Q.astype(np.float64)[:, None, :]
    dist = ((xs - qv) ** 2).sum(-1) if metric == 0 else -(xs * qv).sum(-1)
    order = np.argsort(dist, axis=1, kind="stable")
    return np.take_along_axis(ids, order, 1), np.take_along_axis(dist, order, 1)


def recall_at_k(ids, gt_dist, X, Q, metric=0):
    """Tie-tolerant Recall@k: a returned id counts when its FP64 distance is
    at most the true k-th (1e-9 relative for summation order)."""
    k = gt_dist.shape[1]
    I = ids[:, :k]
    ok = I >= 0
    xs = X[np.maximum(I, 0)].astype(np.float64)
    qv = Q.astype(np.float64)[:, None, :]
    dd = ((xs - qv) ** 2).sum(-1) if metric == 0 else -(xs * qv).sum(-1)
    kth = gt_dist[:, k - 1][:, None]
    return float((ok & (dd <= kth + 1e-9 * np.abs(kth))).sum() / I.size)


def calib_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per dispatch."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n * 4, "dispatches": 3}), flush=True)


def distance_error(ids, dist, gt_dist, Xd64_rows_fn, sample):
    """Returned distances against FP64 recomputation of the returned ids
    (max / mean relative error) and the mean ratio of the j-th returned
    FP64 distance to the true j-th distance (L2 only; 1 = exact)."""
    errs, ratios = [], []
    for j, qi in enumerate(sample):
        ok = ids[qi] >= 0
        dd = Xd64_rows_fn(qi, ids[qi])
        errs.extend((np.abs(dist[qi][ok].astype(np.float64) - dd[ok])
                     / np.maximum(np.abs(dd[ok]), 1e-30)).tolist())
        m = int(ok.sum())
        ratios.extend((dd[:m] / np.maximum(gt_dist[j, :m], 1e-30)).tolist())
    e = np.array(errs) if errs else np.zeros(1)
    return {"max_rel_err": float(e.max()), "mean_rel_err": float(e.mean()),
            "mean_dist_ratio": float(np.mean(ratios)) if ratios else None}


def recall_of(ids, gt_dist, Xd64_rows_fn, sample):
    """Tie-tolerant Recall@k on the sampled queries (see oracle.recall_at_k).
    The returned ids' FP64 distances are summed in a different order than the
    oracle's, so the comparison with the true k-th distance allows 1e-9
    relative (FP64 rounding is ~1e-16; distinct FP32 points differ by far more)."""
    hits = 0
    k = gt_dist.shape[1]
    for j, qi in enumerate(sample):
        kth = gt_dist[j, k - 1]
        dd = Xd64_rows_fn(qi, ids[qi])
        hits += int(np.sum((ids[qi] >= 0) & (dd <= kth + 1e-9 * abs(kth))))
    return hits / float(len(sample) * k)


def main():
    args = parse()
    if args.calib_copy:
        calib_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): the index and the queries of "
              "every workload here fit one MI355X, and sharded multi-GPU search is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batched":
        batched(args)
        return
    if args.mode == "serving":
        serving(args)
        return
    if args.mode == "worstcase":
        worstcase(args)
        return
    if args.mode == "dynamic":
        dynamic(args)
        return
    import torch

    import paper_2505_17368_amd as hn
    import workloads as wl

    dev = torch.device("cuda:0")
    w = wl.WORKLOADS[args.workload]
    t0 = time.time()
    X, Q = wl.make(args.workload, n=args.n, nq=args.nq)
    n, d = X.shape
    nq = Q.shape[0]
    metric = 0 if w["metric"] == "l2" else 1
    log(f"data {n}x{d}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    forms = args.forms.split(",")
    efs = [int(e) for e in args.efs.split(",")]
    k = args.k
    storage_of = {"f32": 0, "bf16": 1, "fp8": 2}
    graph = hn.GRAPH[args.graph]

    # ---- build once (FP32), then the same hierarchy with BF16 / FP8 rows ----
    indexes = {}
    build_s = {}
    torch.cuda.synchronize()
    t = time.time()
    bparams = dict(gram=GRAM[args.gram], degree=args.degree, metric=metric, graph=graph,
                   max_degree=args.max_degree,
                   root_complete_max=args.root_max, sampler=hn.SAMPLER[args.sampler],
                   ef_construction=args.ef_construction, insert_shift=args.insert_shift)
    base = hn.henn_build(Xd, storage=0, **bparams)
    torch.cuda.synchronize()
    build_s["f32"] = time.time() - t
    log(f"build: {build_s['f32']:.2f}s, layers "
        f"{[base.layer_info(i)['size'] for i in range(base.num_layers)]}")
    exported = [base.export_layer(i) for i in range(base.num_layers)]
    for f in forms:
        if f == "f32":
            indexes[f] = base
            continue
        t = time.time()
        indexes[f] = hn.henn_import(Xd, [e[0] for e in exported], [e[1] for e in exported],
                                    storage=storage_of[f], **bparams)
        torch.cuda.synchronize()
        build_s[f] = build_s["f32"] + time.time() - t
    layers_info = [base.layer_info(i) for i in range(base.num_layers)]

    # ---- exact FP64 ground truth of the queries ----
    threads, affinity, nproc = cpu_threads()
    rng = np.random.default_rng(123)
    sample = (np.arange(nq) if args.gt_sample <= 0 or args.gt_sample >= nq
              else np.sort(rng.choice(nq, args.gt_sample, replace=False)))
    t = time.time()
    gt_ids, gt_dist = exact_knn(X, Q[sample], k, metric)
    log(f"exact FP64 ground truth for {len(sample)} queries in {time.time() - t:.1f}s")

    def dist_rows(qi, ids):
        ok = ids >= 0
        out = np.full(ids.shape, np.inf)
        if ok.any():
            xs = X[ids[ok]].astype(np.float64)
            qv = Q[qi].astype(np.float64)
            out[ok] = ((xs - qv) ** 2).sum(1) if metric == 0 else -(xs @ qv)
        return out

    # ---- sweep: recall and single-launch time per (form, ef) ----
    fixed = None
    if args.shape:
        lp, wp, vb, ps = (int(x) for x in args.shape.split(","))
        fixed = {"lanes_per_vec": lp, "waves_per_block": wp, "vis_bits": vb, "persistent": bool(ps)}

    def run(idx, ef, persistent=False, events=None, **kw):
        if fixed is not None:
            return hn.henn_search_batch(idx, Qd, k=k, ef=ef, k_max=k, ef_max=ef, events=events,
                                        lanes_per_vec=fixed["lanes_per_vec"],
                                        waves_per_block=fixed["waves_per_block"],
                                        vis_bits=fixed["vis_bits"],
                                        persistent=fixed["persistent"], **kw)
        return hn.henn_search_batch(idx, Qd, k=k, ef=ef, k_max=k, ef_max=ef,
                                    persistent=persistent, events=events, **kw)

    def time_launches(idx, ef, reps, persistent=False):
        for _ in range(2):
            run(idx, ef, persistent)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            run(idx, ef, persistent)
            e1.record(st)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return np.array(ts)

    sweep = {}
    chosen = {}
    tuned = {}
    # the tuner sees the timed batch itself: the best shape depends on how
    # many query waves the batch puts in flight
    calib = Qd
    for f in forms:
        sweep[f] = []
        for ef in efs:
            # the library's autotuner picks and caches the launch shape
            tuned[(f, ef)] = fixed if fixed is not None else hn.henn_autotune(
                indexes[f], calib, k=k, ef=ef)
            ids, dist = run(indexes[f], ef)
            torch.cuda.synchronize()
            qual = quality(ids.cpu().numpy(), dist.cpu().numpy(), gt_dist, X, Q, sample, metric)
            rec = qual["recall"]
            if fixed is not None:
                ts = time_launches(indexes[f], ef, 5)
                best, pers = float(np.median(ts)), fixed["persistent"]
            else:
                # the persistent launch only when it is clearly faster: at equal
                # times the plain grid's steady state is the better one
                ts = time_launches(indexes[f], ef, 9)
                tp = time_launches(indexes[f], ef, 9, persistent=True)
                pers = float(np.median(tp)) < 0.98 * float(np.median(ts))
                best = float(np.median(tp)) if pers else float(np.median(ts))
            qps = nq / (best / 1e3)
            sweep[f].append({"ef": ef, "recall": round(rec, 4),
                             "recall_ci95": round(qual["recall_ci95"], 4),
                             "ms": round(best, 3),
                             "qps": round(qps, 1), "persistent": pers,
                             "shape": tuned[(f, ef)],
                             "max_rel_dist_err": round(qual["max_rel_err"], 9),
                             "mean_dist_ratio": round(qual["mean_dist_ratio"], 6)
                             if qual["mean_dist_ratio"] is not None else None})
            log(f"{f} ef={ef}: recall {rec:.4f} +- {qual['recall_ci95']:.4f}  {best:.3f} ms  "
                f"{qps:,.0f} QPS (persistent {pers})")
            if rec >= args.target_recall and f not in chosen:
                chosen[f] = sweep[f][-1]
        if f not in chosen:
            chosen[f] = max(sweep[f], key=lambda r: r["recall"])
    meets = {f: c for f, c in chosen.items() if c["recall"] >= args.target_recall}
    pool = meets if meets else chosen
    head_form = max(pool, key=lambda f: pool[f]["qps"])
    head = chosen[head_form]
    idx = indexes[head_form]
    ef = head["ef"]
    pers = head["persistent"]

    # ---- counts of the algorithmic byte model: the same search with an exact
    # visited set, which evaluates each node once per layer as the method does
    _, _, cnt = hn.henn_search_batch(idx, Qd, k=k, ef=ef, k_max=k, ef_max=ef,
                                     with_counters=True, exact_visited=True)
    torch.cuda.synchronize()
    cnt = cnt.cpu().numpy().astype(np.float64)

    # ---- CPU baseline: the oracle's search on the same index (host cores) ----
    cpu = None
    if not args.no_cpu:
        from oracle import henn_oracle as ho
        ids_l = [e[0] for e in exported]
        adj_l = [e[1] for e in exported]
        oidx = ho.index_from_arrays(X, metric, ids_l, adj_l,
                                    root_complete=args.root_max > 0 and len(ids_l) >= 2)
        # grow the sample until the oracle has worked ~cpu_seconds
        m = min(nq, 256)
        done, el = 0, 0.0
        while True:
            sub = Q[done % nq: done % nq + m] if done % nq + m <= nq else Q[:m]
            t = time.time()
            ho.search(oidx, sub, k, ef, 1, threads=threads)
            el += time.time() - t
            done += len(sub)
            if el >= args.cpu_seconds or done >= 64 * nq:
                break
            m = min(nq, m * 2)
        # one thread, query by query, on the first 1,000 queries
        n1 = min(nq, 1000)
        lat = np.empty(n1)
        t = time.time()
        for i in range(n1):
            t0 = time.perf_counter()
            ho.search(oidx, Q[i:i + 1], k, ef, 1, threads=1)
            lat[i] = time.perf_counter() - t0
        el1 = time.time() - t
        cpu = {"value": round(done / el, 2), "unit": "queries/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{done} oracle searches over the {nq} workload queries taken in "
                         f"order and repeated (same index, ef={ef}, "
                         f"k={k}), FP64 C oracle, {threads} threads, {el:.1f}s",
               "nproc": nproc, "affinity_cpus": affinity,
               "threads_note": "threads = the affinity mask, at most 16 (the host's CPU "
                               "share per GPU)",
               "value_1_thread": round(n1 / el1, 2),
               "sample_1_thread": f"the first {n1} queries on one thread, one call each, "
                                  f"{el1:.1f}s",
               "latency_1_thread_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                                       "max": round(float(lat.max()) * 1e3, 3),
                                       "note": "per call, including the binding's overhead"},
               "cpu_model": _cpu_model()}
        log(f"cpu baseline {cpu['value']} QPS on {threads} threads, "
            f"{cpu['value_1_thread']} QPS on one")

    # ---- timed region: exactly --steps batched searches ----
    # a workspace and the outputs are allocated once, outside the timed region
    wsb = hn.workspace_size(idx, nq, k=k, ef=ef, k_max=k, ef_max=ef,
                            persistent=pers if fixed is None else fixed["persistent"])
    wsp = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    o_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    o_dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    tkw = dict(workspace=wsp, out_ids=o_ids, out_dist=o_dist)
    for _ in range(args.warmup):
        run(idx, ef, pers, **tkw)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a_, b_ in kev:  # materialise the events; the library re-records them
        a_.record(st)
        b_.record(st)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for (e0, e1), ke in zip(evs, kev):
        e0.record(st)
        run(idx, ef, pers, events=ke, **tkw)
        e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    search_ms = np.array([a_.elapsed_time(b_) for a_, b_ in kev])
    ms_per_step = wall * 1e3 / args.steps
    value = nq * args.steps / wall
    timed_ok = quality(o_ids.cpu().numpy(), o_dist.cpu().numpy(), gt_dist, X, Q, sample,
                       metric)["recall"]

    # ---- roofline of the search kernel (HBM bound, algorithmic bytes) ----
    b = {"f32": 4, "bf16": 2, "fp8": 1}[head_form]
    bs = 4 if head_form == "fp8" else 0
    src = cnt
    # the root's exhaustive scan runs in its own kernels; the roofline is that
    # of the dominant kernel, k_search: the layers below the root, each
    # evaluation a row gather, each expansion an adjacency row
    root_n = layers_info[-1]["size"] if args.root_max > 0 and len(layers_info) >= 2 else 0
    evals = src[:, 1].mean() - root_n
    exps = src[:, 0].mean()
    n_rr = 0 if head_form == "f32" else min(max(ef, k), 4 * k)
    deg = layers_info[0]["degree"]
    bytes_q = evals * (d * b + bs) + exps * deg * 4 + n_rr * d * 4 + d * 4 + k * 8
    kernel_ms = float(np.mean(search_ms))
    achieved = bytes_q * nq / (kernel_ms / 1e3) / 1e9
    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    # copy-calibrated), valid only while the kernel source is unchanged and
    # for the same workload / form / beam width
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "k_search_traffic.json")
    if os.path.exists(tpath):
        from paper_2505_17368_amd.kernel_hash import search_kernel_hash
        h = search_kernel_hash()
        for tr in json.load(open(tpath)).get("entries", []):
            if (tr.get("source_hash") == h and tr.get("workload") == args.workload
                    and tr.get("form") == head_form and tr.get("ef") == ef
                    and tr.get("graph") == args.graph and tr.get("degree") == args.degree
                    and tr.get("max_degree") == args.max_degree):
                traffic = round(tr["fetch_bytes"] + tr["write_bytes"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_query": round(bytes_q, 1), "evals_per_query": round(evals, 1),
                "expansions_per_query": round(exps, 1), "kernel": "k_search",
                "kernel_ms": round(kernel_ms, 4),
                "count_source": "exact-visited search"}

    dtype_of = {"f32": "f32", "bf16": "bf16 storage, f32 accumulate",
                "fp8": "fp8_e4m3 storage, f16 difference, f32 accumulate"}
    out = {
        "metric": "QPS at recall@10>=0.95, n=1M d=128; BF16/FP8 vs FP32 form; p99 ms",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of[head_form],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "nq": nq, "k": k, "ef": ef,
                   "form": head_form, "storage": head_form, "persistent": pers,
                   "graph": args.graph, "sampler": args.sampler, "degree": args.degree,
                   "max_degree": args.max_degree,
                   **({"ef_construction": args.ef_construction,
                       "insert_shift": args.insert_shift} if args.graph == "nsw" else {}),
                   "root_complete_max": args.root_max, "metric": w["metric"]},
        "recall_at_10": head["recall"],
        "recall_ci95": head["recall_ci95"],
        "recall_queries": int(len(sample)),
        "recall_timed_run": round(timed_ok, 4),
        "p50_ms": round(float(np.percentile(kms, 50)), 4),
        "p99_ms": round(float(np.percentile(kms, 99)), 4),
        "forms": {f: {**chosen[f], "build_s": round(build_s[f], 2)} for f in forms},
        "sweep": sweep,
        "layers": [li["size"] for li in layers_info],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if not args.no_serve:
        # per-request beam widths: the pick and the next two grid points
        pos = efs.index(ef)
        ef_choices = tuple(efs[pos:pos + 3]) if pos + 3 <= len(efs) else tuple(efs[-3:])
        out["serving"] = serving_experiment(hn, indexes[head_form], Q, gt_dist, dist_rows,
                                            sample, args, ef_choices=ef_choices)
    for f in forms:
        indexes[f].free()
    base.free()
    if not args.no_adversarial and args.workload == "gmm100_1M_d128" and args.n is None:
        out["adversarial"] = adversarial_experiment(hn, args, threads)
    print(json.dumps(out), flush=True)


def adversarial_experiment(hn, args, threads, wname="curve_1M_d96", storage="bf16"):
    """The adversarial-layout workload: 1M x 96 points along a curve whose
    gaps shrink as 0.5^(i mod 40) (Sec. 4.2's skewed regime), 10,000 queries
    near the dense end of random periods; BF16 traversal rows and an FP32
    re-rank of 4k = 40 candidates, k = 10.  The smallest swept beam width
    whose Recall@10 (all queries, exact FP64 ground truth) reaches the target
    is timed; the roofline of k_search uses the counts of the same search
    with an exact visited set."""
    import torch
    import workloads as wl
    dev = torch.device("cuda:0")
    k = 10
    X, Q = wl.make(wname)
    n, d = X.shape
    nq = Q.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    bp = dict(gram=GRAM[args.gram], degree=args.degree, metric=0, graph=hn.GRAPH[args.graph],
              max_degree=args.max_degree, root_complete_max=args.root_max)
    torch.cuda.synchronize()
    t = time.time()
    base = hn.henn_build(Xd, storage=0, **bp)
    torch.cuda.synchronize()
    build_s = time.time() - t
    ex = [base.export_layer(i) for i in range(base.num_layers)]
    sizes = [len(e[0]) for e in ex]
    st_code = {"f32": 0, "bf16": 1, "fp8": 2}[storage]
    idx = hn.henn_import(Xd, [e[0] for e in ex], [e[1] for e in ex], storage=st_code, **bp)
    t = time.time()
    sample = np.arange(nq)
    _, gt_dist = exact_knn(X, Q, k, 0)
    log(f"adversarial: build {build_s:.1f}s, layers {sizes}, ground truth "
        f"{time.time() - t:.1f}s")
    sweep, pick = [], None
    for ef in [int(e) for e in args.efs.split(",")]:
        hn.henn_autotune(idx, Qd, k=k, ef=ef)
        ids, dist = hn.henn_search_batch(idx, Qd, k=k, ef=ef)
        torch.cuda.synchronize()
        qual = quality(ids.cpu().numpy(), dist.cpu().numpy(), gt_dist, X, Q, sample, 0)
        sweep.append({"ef": ef, "recall": round(qual["recall"], 4)})
        log(f"adversarial ef={ef}: recall {qual['recall']:.4f}")
        if qual["recall"] >= args.target_recall:
            pick = (ef, qual)
            break
    if pick is None:
        idx.free()
        base.free()
        return {"workload": wname, "sweep": sweep, "reached_target": False}
    ef, qual = pick
    st = torch.cuda.current_stream()
    for _ in range(3):
        hn.henn_search_batch(idx, Qd, k=k, ef=ef)
    torch.cuda.synchronize()
    ts, ks = [], []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(st)
        k1.record(st)
        e0.record(st)
        hn.henn_search_batch(idx, Qd, k=k, ef=ef, events=(k0, k1))
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
        ks.append(k0.elapsed_time(k1))
    ms, kms = float(np.median(ts)), float(np.mean(ks))
    _, _, cnt = hn.henn_search_batch(idx, Qd, k=k, ef=ef, with_counters=True,
                                     exact_visited=True)
    cnt = cnt.cpu().numpy().astype(np.float64)
    root_n = sizes[-1] if args.root_max > 0 and len(sizes) >= 2 else 0
    evals = cnt[:, 1].mean() - root_n
    exps = cnt[:, 0].mean()
    deg = ex[0][1].shape[1]
    bytes_q = evals * d * 2 + exps * deg * 4 + min(ef, 4 * k) * d * 4 + d * 4 + k * 8
    achieved = bytes_q * nq / (kms / 1e3) / 1e9
    idx.free()
    base.free()
    return {"workload": wname, "n": n, "d": d, "nq": nq, "k": k, "storage": storage,
            "dtype": "bf16 storage, f32 accumulate", "rerank": 4 * k, "ef": ef,
            "recall_at_10": round(qual["recall"], 4), "recall_ci95": round(qual["recall_ci95"], 4),
            "qps": round(nq / (ms / 1e3), 1), "ms_per_batch": round(ms, 4),
            "max_rel_dist_err": round(qual["max_rel_err"], 9),
            "mean_dist_ratio": round(qual["mean_dist_ratio"], 6),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "kernel": "k_search", "kernel_ms": round(kms, 4),
                         "bytes_per_query": round(bytes_q, 1),
                         "evals_per_query": round(evals, 1),
                         "expansions_per_query": round(exps, 1),
                         "count_source": "exact-visited search"},
            "build_s": round(build_s, 2), "layers": sizes, "sweep": sweep,
            "graph": args.graph, "degree": args.degree, "max_degree": args.max_degree,
            "root_complete_max": args.root_max}


def serving_experiment(hn, idx, Q, gt_dist, dist_rows, sample, args, k_choices=(10, 50),
                       ef_choices=(128, 192, 256), fracs=(0.25, 0.5, 0.75)):
    """Continuous batching under Poisson arrivals: each request has its own
    k (from k_choices, seed 6) and beam width (from ef_choices, seed 7);
    first the saturated throughput (every request already queued when the
    clock starts: the server never waits for work), then the given fractions
    of it as arrival rates, whose requests are submitted inside the timed
    loop as they arrive.  Latency = completion observed by the host -
    arrival.  The batch form's QPS on the same requests (per-request k and
    ef in one persistent launch) is reported beside the saturated rate."""
    import workloads as wl
    nq = Q.shape[0]
    # requests cycle through the workload's queries (request i asks query i mod nq)
    n_req = args.serve_requests
    rk = np.random.default_rng(6).choice(list(k_choices), size=n_req).astype(np.int32)
    ref = np.random.default_rng(7).choice(list(ef_choices), size=n_req).astype(np.int32)
    k_max, ef_max = int(max(k_choices)), int(max(ef_choices))
    qs = Q[np.arange(n_req) % nq]
    tags = np.arange(n_req, dtype=np.int64)

    def run(arrivals):
        srv = hn.Server(idx, max_slots=args.serve_slots, pool_bytes=args.serve_pool_mb << 20,
                        k_max=k_max, ef_max=ef_max, steps_per_tick=args.serve_steps)
        done_t = np.zeros(n_req)
        got_ids = np.full((n_req, k_max), -1, dtype=np.int32)
        nxt, ndone, ticks = 0, 0, 0
        if not arrivals.any():  # saturated: the whole backlog is queued first
            srv.submit_batch(qs, rk, ref, tags)
            nxt = n_req
        # the harness's own garbage collection stays out of the latencies
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        while ndone < n_req:
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arrivals, now, side="right"))
            if j > nxt:
                srv.submit_batch(qs[nxt:j], rk[nxt:j], ref[nxt:j], tags[nxt:j])
                nxt = j
            srv.tick()
            ticks += 1
            tg, ids, _ = srv.poll()
            if len(tg):
                tnow = time.perf_counter() - t0
                done_t[tg] = tnow
                got_ids[tg] = ids
                ndone += len(tg)
        gc.enable()
        st = srv.stats()
        srv.close()
        lat = (done_t - arrivals) * 1e3
        span = done_t.max() - arrivals.min()
        return {"qps": round(n_req / span, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "max_ms": round(float(lat.max()), 3), "ticks": ticks,
                "max_active": int(st["max_active"])}, got_ids

    # one short run first, so that no timed tick pays for first use (code
    # loading, first touch of the state pool)
    warm = min(n_req, 256)
    srv = hn.Server(idx, max_slots=args.serve_slots, pool_bytes=args.serve_pool_mb << 20,
                    k_max=k_max, ef_max=ef_max, steps_per_tick=args.serve_steps)
    srv.submit_batch(qs[:warm], rk[:warm], ref[:warm], tags[:warm])
    left = warm
    while left > 0:
        srv.tick()
        left -= len(srv.poll()[0])
    srv.close()
    sat, ids = run(np.zeros(n_req))
    # the batch form on the same requests (per-request k and ef), for scale
    import torch
    Qs = torch.from_numpy(np.ascontiguousarray(qs)).cuda()
    ka = torch.from_numpy(rk).cuda()
    ea = torch.from_numpy(ref).cuda()
    bkw = dict(k_arr=ka, ef_arr=ea, k_max=k_max, ef_max=ef_max, persistent=True)
    hn.henn_search_batch(idx, Qs, **bkw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        hn.henn_search_batch(idx, Qs, **bkw)
    torch.cuda.synchronize()
    batch_qps = 3 * n_req / (time.perf_counter() - t)
    sat["batch_same_mix_qps"] = round(batch_qps, 1)
    sat["serving_over_batch"] = round(sat["qps"] / batch_qps, 3)
    del Qs, ka, ea
    # recall over the first request of each sampled query
    in_sample = [j for j, qi in enumerate(sample) if qi < min(n_req, nq)]
    rec = recall_of(ids[:min(n_req, nq), :10], gt_dist[in_sample], dist_rows,
                    np.asarray(sample)[in_sample]) if in_sample else None
    # one short run at the lowest rate first (not reported), so that no
    # timed Poisson run pays for first use of its code paths and buffers
    warm_n = min(n_req, 10000)
    warm_arr = wl.poisson_arrivals(warm_n, min(fracs) * sat["qps"], seed=4)
    warm_arr -= warm_arr[0]
    srv = hn.Server(idx, max_slots=args.serve_slots, pool_bytes=args.serve_pool_mb << 20,
                    k_max=k_max, ef_max=ef_max, steps_per_tick=args.serve_steps)
    t0, nxt, left = time.perf_counter(), 0, warm_n
    while left > 0:
        j = int(np.searchsorted(warm_arr, time.perf_counter() - t0, side="right"))
        if j > nxt:
            srv.submit_batch(qs[nxt:j], rk[nxt:j], ref[nxt:j], tags[nxt:j])
            nxt = j
        srv.tick()
        left -= len(srv.poll()[0])
    srv.close()
    levels = []
    for frac in fracs:
        rate = frac * sat["qps"]
        arr = wl.poisson_arrivals(n_req, rate, seed=5)
        arr -= arr[0]
        r, _ = run(arr)
        r["offered_qps"] = round(rate, 1)
        levels.append(r)
        log(f"serving at {rate:,.0f} QPS offered: {r}")
    log(f"serving saturated: {sat}, recall@10 {rec}")
    return {"requests": n_req, "k": list(k_choices), "ef": list(ef_choices),
            "steps_per_tick": args.serve_steps, "slots": args.serve_slots,
            "pool_mb": args.serve_pool_mb, "saturated": sat, "recall_at_10": rec,
            "poisson": levels}



def batched(args):
    """Batched mixed-request form: every query carries its own k in
    {1, 10, 100} and beam width in {32, 64, 128} (ef_eff = max(ef, k)); the
    whole batch runs as one persistent launch captured in a hipGraph, with
    the launch shape chosen by the library's autotuner."""
    import torch

    import paper_2505_17368_amd as hn
    import workloads as wl

    wname = args.workload if args.workload != "gmm100_1M_d128" else "gmm1000_10M_d128"
    w = wl.WORKLOADS[wname]
    dev = torch.device("cuda:0")
    t0 = time.time()
    X, Q = wl.make(wname, n=args.n, nq=args.nq)
    n, d = X.shape
    nq = Q.shape[0]
    metric = 0 if w["metric"] == "l2" else 1
    ks, efs = wl.mixed_requests(nq)
    log(f"data {n}x{d}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    bp = dict(gram=GRAM[args.gram], degree=args.degree, metric=metric, graph=hn.GRAPH[args.graph],
              sampler=hn.SAMPLER[args.sampler], ef_construction=args.ef_construction,
              insert_shift=args.insert_shift,
              max_degree=args.max_degree, root_complete_max=args.root_max)
    torch.cuda.synchronize()
    t = time.time()
    base = hn.henn_build(Xd, storage=0, **bp)
    torch.cuda.synchronize()
    build_s = time.time() - t
    sizes = [base.layer_info(i)["size"] for i in range(base.num_layers)]
    log(f"build {build_s:.1f}s, layers {sizes}")
    st_code = {"f32": 0, "bf16": 1, "fp8": 2}[args.storage]
    if st_code:
        ex = [base.export_layer(i) for i in range(base.num_layers)]
        idx = hn.henn_import(Xd, [e[0] for e in ex], [e[1] for e in ex], storage=st_code, **bp)
        base.free()
        del ex
    else:
        idx = base
    k_d = torch.from_numpy(ks).to(dev)
    ef_d = torch.from_numpy(efs).to(dev)
    calib = min(nq, 16384)
    shape = hn.henn_autotune(idx, Qd[:calib], k=10, ef=128, k_arr=k_d[:calib],
                             ef_arr=ef_d[:calib], k_max=100, ef_max=128)
    log(f"autotuned shape {shape}")
    g = hn.SearchGraph(idx, Qd.clone(), k=10, ef=128, k_arr=k_d, ef_arr=ef_d, k_max=100,
                       ef_max=128, persistent=True)
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        g.launch()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kms = np.array([a.elapsed_time(b) for a, b in evs])
    ids = g.ids.cpu().numpy()
    # recall per k class on a sample, against exact FP64 brute force
    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(nq, min(args.gt_sample, nq), replace=False))
    t = time.time()
    gt_ids, gt_dist = exact_knn(X, Q[sample], 100, metric) if len(sample) else (None, None)
    log(f"exact ground truth (k=100) for {len(sample)} queries in {time.time() - t:.1f}s")
    per_k = {}
    for kk in (1, 10, 100):
        sel = [j for j, qi in enumerate(sample) if ks[qi] == kk]
        hits = 0
        for j in sel:
            qi = sample[j]
            row = ids[qi, :kk]
            ok = row >= 0
            xs = X[row[ok]].astype(np.float64)
            qv = Q[qi].astype(np.float64)
            dd = ((xs - qv) ** 2).sum(1) if metric == 0 else -(xs @ qv)
            kth = gt_dist[j, kk - 1]
            hits += int(np.sum(dd <= kth + 1e-9 * abs(kth)))
        per_k[f"k={kk}"] = round(hits / max(1, len(sel) * kk), 4) if sel else None
    g.free()
    idx.free()
    out = {
        "metric": "batched mixed-request QPS (one persistent hipGraph launch)",
        "value": round(nq * args.steps / wall, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 storage, f32 accumulate",
                  "fp8": "fp8_e4m3 storage, f16 difference, f32 accumulate"}[args.storage],
        "data": "synthetic",
        "config": {"workload": wname, "n": n, "d": d, "nq": nq, "storage": args.storage,
                   "k": [1, 10, 100], "ef": [32, 64, 128], "graph": args.graph,
                   "sampler": args.sampler,
                   "max_degree": args.max_degree, "root_complete_max": args.root_max},
        "p50_ms": round(float(np.percentile(kms, 50)), 3),
        "p99_ms": round(float(np.percentile(kms, 99)), 3),
        "recall_by_k": per_k, "build_s": round(build_s, 1), "layers": sizes, "shape": shape,
    }
    print(json.dumps(out), flush=True)


def serving(args):
    """Serving form on the embedding-retrieval workload (5M x 768 unit
    vectors, inner product, BF16 rows with an FP32 re-rank): build once,
    take as per-request beam widths the three smallest sweep points at or
    above the first one reaching the recall target at k = 10, then run
    continuous batching saturated and at fractions of that rate under
    Poisson arrivals, with k in {10, 50} per request."""
    import torch

    import paper_2505_17368_amd as hn
    import workloads as wl

    wname = args.workload if args.workload != "gmm100_1M_d128" else "spectral_5M_d768"
    w = wl.WORKLOADS[wname]
    dev = torch.device("cuda:0")
    t0 = time.time()
    X, Q = wl.make(wname, n=args.n, nq=args.nq)
    n, d = X.shape
    nq = Q.shape[0]
    metric = 0 if w["metric"] == "l2" else 1
    log(f"data {n}x{d}, {nq} queries in {time.time() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    bp = dict(gram=GRAM[args.gram], degree=args.degree, metric=metric, graph=hn.GRAPH[args.graph],
              sampler=hn.SAMPLER[args.sampler], ef_construction=args.ef_construction,
              insert_shift=args.insert_shift,
              max_degree=args.max_degree, root_complete_max=args.serve_root_max)
    torch.cuda.synchronize()
    t = time.time()
    base = hn.henn_build(Xd, storage=0, **bp)
    torch.cuda.synchronize()
    build_s = time.time() - t
    sizes = [base.layer_info(i)["size"] for i in range(base.num_layers)]
    fallback = [base.layer_info(i)["fallback_rows"] for i in range(base.num_layers)]
    log(f"build {build_s:.1f}s, layers {sizes}, exact-fallback rows {fallback}")
    st_code = {"f32": 0, "bf16": 1, "fp8": 2}[args.storage]
    if st_code:
        ex = [base.export_layer(i) for i in range(base.num_layers)]
        idx = hn.henn_import(Xd, [e[0] for e in ex], [e[1] for e in ex], storage=st_code, **bp)
        base.free()
        del ex
    else:
        idx = base

    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(nq, min(args.gt_sample, nq), replace=False))
    t = time.time()
    _, gt_dist = exact_knn(X, Q[sample], 10, metric)
    log(f"exact ground truth for {len(sample)} queries in {time.time() - t:.1f}s")

    def dist_rows(qi, ids):
        ok = ids >= 0
        out = np.full(ids.shape, np.inf)
        if ok.any():
            xs = X[ids[ok]].astype(np.float64)
            qv = Q[qi].astype(np.float64)
            out[ok] = ((xs - qv) ** 2).sum(1) if metric == 0 else -(xs @ qv)
        return out

    efs = [int(e) for e in args.efs.split(",")]
    sweep = []
    chosen = None
    for ef in efs:
        hn.henn_autotune(idx, Qd, k=10, ef=ef)
        ids, _ = hn.henn_search_batch(idx, Qd, k=10, ef=ef)
        torch.cuda.synchronize()
        rec = recall_of(ids.cpu().numpy(), gt_dist, dist_rows, sample)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            hn.henn_search_batch(idx, Qd, k=10, ef=ef)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        sweep.append({"ef": ef, "recall": round(rec, 4), "batch_qps": round(nq / (ms / 1e3), 1)})
        log(f"ef={ef}: recall@10 {rec:.4f}, batched {nq / (ms / 1e3):,.0f} QPS")
        if chosen is None and rec >= args.target_recall:
            chosen = ef
    if chosen is None:
        chosen = efs[-1]
    pos = efs.index(chosen)
    ef_choices = tuple(efs[pos:pos + 3]) if pos + 3 <= len(efs) else tuple(efs[-3:])
    log(f"per-request beam widths {ef_choices}")
    res = serving_experiment(hn, idx, Q, gt_dist, dist_rows, list(sample), args,
                             k_choices=(10, 50), ef_choices=ef_choices,
                             fracs=(0.1, 0.3, 0.5, 0.7, 0.9))
    idx.free()
    sat = res["saturated"]
    out = {
        "metric": "serving QPS (continuous batching, saturated) with Poisson-load p50/p99",
        "value": sat["qps"], "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": wname, "n": n, "d": d, "nq": nq, "metric": w["metric"],
                   "storage": args.storage, "graph": args.graph, "sampler": args.sampler,
                   "max_degree": args.max_degree, "root_complete_max": args.serve_root_max},
        "build_s": round(build_s, 1), "layers": sizes, "fallback_rows": fallback,
        "sweep": sweep, "serving": res,
    }
    print(json.dumps(out), flush=True)


def hits_curve(ranks, kmax):
    """Average hits of the recall-bound experiment (App. G.4): for k = 1 ..
    kmax, the fraction of greedy searches whose result is among the k
    nearest points of its query (ranks: 1 = the nearest)."""
    r = np.asarray(ranks).ravel()
    return np.array([(r <= k).mean() for k in range(1, kmax + 1)]) if r.size else np.zeros(kmax)


def recall_bound(ranks, delta):
    """rho_delta of Sec. 3 (recall bound): the smallest k such that the
    greedy result lies among the k nearest points with probability at least
    delta, the probability taken as the fraction of the searches observed."""
    r = np.sort(np.asarray(ranks).ravel())
    if r.size == 0:
        raise ValueError("no searches")
    return int(r[int(np.ceil(delta * r.size)) - 1])


def ranks_of(Xd, Qd, got):
    """Rank of each query's result among all points (1 = nearest): one plus
    the points strictly closer than it, squared L2 in FP64 on the GPU."""
    import torch
    X64 = Xd.double()
    xn = (X64 * X64).sum(1)
    out = np.empty(Qd.shape[0], np.int64)
    g_all = torch.from_numpy(np.asarray(got)).to(Xd.device, torch.int64)
    for s in range(0, Qd.shape[0], 256):
        q = Qd[s:s + 256].double()
        dd = xn[None, :] - 2.0 * (q @ X64.T)
        mine = dd.gather(1, g_all[s:s + 256, None])
        out[s:s + 256] = ((dd < mine).sum(1) + 1).cpu().numpy()
    return out


def worstcase(args):
    """The paper's synthetic worst-case study (Sec. 4.2 "Synthetic Dataset",
    "Number of Hops"; App. G.4 recall bounds) on the GPU path.

    Hops and query time: HENN with verified eps-net layers (Eq. (1) with a
    small c0, so that the ring check of App. B.1 rejects samples), the same
    with Alg. 3 halving layers, and random layers (every ring vacuous: the
    HNSW-style hierarchy), on skewed exponential data (``expskew``), NSW
    graphs (App. B.2), the same build seeds.  Per build, Alg. 4 greedy
    queries (k = 1, ef = 1) give the hops (expansions over all layers) and
    each query's time on the device clock; "worst case" is the maximum over
    the queries and the runs, as in the paper.  The n = 50,000, d = 32
    configurations also sweep ef at k = 10 for Recall@10.

    Recall bound: rho_0.9 of one navigation graph (kNN or NSW over all n
    points), per its definition in Sec. 3: greedy search on that graph alone
    from a start drawn uniformly per run (a two-layer index whose upper
    layer is the start), the rank of the result among all points, the hits
    curve pooled over --wc-rho-runs runs with fresh data, queries and start."""
    import torch
    import paper_2505_17368_amd as hn
    import workloads as wl
    hn.load_library()
    dev = torch.device("cuda:0")
    nq, runs, lam0 = args.wc_nq, args.wc_runs, args.wc_lam
    configs = [(n, d, lam0) for d in (16, 32) for n in (1 << 14, 1 << 16, 1 << 18, 1 << 20)]
    configs += [(1 << 16, d, lam0) for d in (8, 64, 128)]
    recall_configs = [(50_000, 32, lam) for lam in (4.0, 32.0, 256.0)]
    efs = (8, 16, 32, 64, 128)
    study = []
    st = torch.cuda.current_stream()

    def timed(idx, Qd, **kw):
        hn.henn_search_batch(idx, Qd, **kw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            hn.henn_search_batch(idx, Qd, **kw)
            e1.record(st)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    parts = set(args.wc_parts.split(","))
    for n, d, lam in (configs + recall_configs if "hops" in parts else []):
        t0 = time.time()
        X = wl.expskew(n, d, lam, seed=0)
        Q = wl.expskew(nq, d, lam, seed=1)
        Xd, Qd = torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev)
        gt10 = exact_knn(X, Q, 10, 0)[1] if (n, d, lam) in recall_configs else None
        entry = {"n": n, "d": d, "lam": lam}
        for variant in ("eps_net", "halving", "random"):
            per_run = []
            for run in range(runs):
                bp = dict(degree=16, max_degree=32, graph=hn.GRAPH["nsw"], ef_construction=256,
                          seed=1000 + run)
                if variant == "random":
                    bp["eps_override"] = 2.0          # every ring vacuous: random layers
                else:
                    bp["c0"] = args.wc_c0d / d
                    if variant == "halving":
                        bp["sampler"] = hn.SAMPLER["halving"]
                idx = hn.henn_build(Xd, **bp)
                info = [idx.layer_info(i) for i in range(1, idx.num_layers)]
                ids, _, cnt, qns = hn.henn_search_batch(idx, Qd, k=1, ef=1, with_counters=True,
                                                        with_times=True)
                torch.cuda.synchronize()
                hops = cnt[:, 0].cpu().numpy()
                qus = qns.cpu().numpy() / 1e3
                rank = ranks_of(Xd, Qd, ids[:, 0].cpu().numpy())
                r = {"mean_hops": float(hops.mean()), "max_hops": int(hops.max()),
                     "query_us_p50": round(float(np.percentile(qus, 50)), 2),
                     "query_us_p99": round(float(np.percentile(qus, 99)), 2),
                     "query_us_max": round(float(qus.max()), 2),
                     "greedy_ms": timed(idx, Qd, k=1, ef=1),
                     "exact_nn": float((rank == 1).mean()),
                     "layers": [x["size"] for x in info],
                     "attempts": [x["attempts"] for x in info],
                     "status": [x["status"] for x in info]}
                if gt10 is not None:
                    r["sweep"] = []
                    for ef in efs:
                        ids10, _ = hn.henn_search_batch(idx, Qd, k=10, ef=ef)
                        torch.cuda.synchronize()
                        rec = recall_at_k(ids10.cpu().numpy(), gt10, X, Q)
                        ms = timed(idx, Qd, k=10, ef=ef)
                        r["sweep"].append({"ef": ef, "recall": round(rec, 4),
                                           "qps": round(nq / (ms / 1e3), 1)})
                per_run.append(r)
                idx.free()
            entry[variant] = {
                "worst_mean_hops": max(r["mean_hops"] for r in per_run),
                "worst_max_hops": max(r["max_hops"] for r in per_run),
                "worst_query_us": max(r["query_us_max"] for r in per_run),
                "worst_query_us_p99": max(r["query_us_p99"] for r in per_run),
                "worst_greedy_ms": max(r["greedy_ms"] for r in per_run),
                "runs": per_run}
        e, hv, r = entry["eps_net"], entry["halving"], entry["random"]
        log(f"n={n} d={d} lam={lam:g}: worst mean hops {e['worst_mean_hops']:.1f} (eps-net) / "
            f"{hv['worst_mean_hops']:.1f} (halving) / {r['worst_mean_hops']:.1f} (random); "
            f"worst max hops {e['worst_max_hops']} / {hv['worst_max_hops']} / "
            f"{r['worst_max_hops']}; worst query {e['worst_query_us']:.1f} / "
            f"{hv['worst_query_us']:.1f} / {r['worst_query_us']:.1f} us; "
            f"{time.time() - t0:.1f}s")
        study.append(entry)
        del Xd, Qd

    # ---- recall bound rho_0.9 of one navigation graph (Sec. 3, App. G.4) ----
    rho = []
    rho_q = args.wc_rho_nq
    for graph in (("knn", "nsw") if "rho" in parts else ()):
        for lam in (1.0, 32.0):
            for n in (10_000, 50_000, 200_000):
                t0 = time.time()
                ranks, per_run = [], []
                for run in range(args.wc_rho_runs):
                    X = wl.expskew(n, 32, lam, seed=10_000 + run)
                    Q = wl.expskew(rho_q, 32, lam, seed=20_000 + run)
                    Xd, Qd = torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev)
                    bp = dict(degree=16, max_degree=32, graph=hn.GRAPH[graph], max_layers=0,
                              ef_construction=256, seed=run)
                    g = hn.henn_build(Xd, **bp)
                    _, adj = g.export_layer(0)
                    g.free()
                    start = int(np.random.default_rng(30_000 + run).integers(n))
                    two = hn.henn_import(Xd, [None, np.array([start], np.int32)],
                                         [adj, -np.ones((1, adj.shape[1]), np.int32)],
                                         degree=16, max_degree=32, graph=hn.GRAPH[graph])
                    ids, _ = hn.henn_search_batch(two, Qd, k=1, ef=1)
                    torch.cuda.synchronize()
                    two.free()
                    rk = ranks_of(Xd, Qd, ids[:, 0].cpu().numpy())
                    ranks.append(rk)
                    per_run.append(recall_bound(rk, 0.9))
                    del Xd, Qd
                ranks = np.concatenate(ranks)
                hc = hits_curve(ranks, 100)
                row = {"graph": graph, "n": n, "d": 32, "lam": lam, "runs": args.wc_rho_runs,
                       "queries_per_run": rho_q, "rho_0.9": recall_bound(ranks, 0.9),
                       "hits": {f"k={k}": round(float(hc[k - 1]), 4) for k in (1, 5, 10, 15, 50)},
                       "rho_0.9_per_run": {"min": int(min(per_run)),
                                           "median": float(np.median(per_run)),
                                           "max": int(max(per_run))}}
                rho.append(row)
                log(f"recall bound {graph} n={n} lam={lam:g}: rho_0.9 {row['rho_0.9']} "
                    f"(per run {row['rho_0.9_per_run']}), hits@1 {row['hits']['k=1']}, "
                    f"{time.time() - t0:.1f}s")

    ratios = [x["random"]["worst_mean_hops"] / x["eps_net"]["worst_mean_hops"]
              for x in study if (x["n"], x["d"], x["lam"]) in configs]
    ratios_h = [x["random"]["worst_mean_hops"] / x["halving"]["worst_mean_hops"]
                for x in study if (x["n"], x["d"], x["lam"]) in configs]

    def gmean(v):
        return round(float(np.exp(np.mean(np.log(v)))), 4) if v else None
    out = {
        "metric": "worst-case Alg. 4 hops, random layers / eps-net layers (geometric mean over "
                  "the n and d sweeps)",
        "value": gmean(ratios), "unit": "ratio",
        "halving_ratio": gmean(ratios_h),
        "n_gpus": 1, "steps": runs, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "expskew", "nq": nq, "runs": runs, "lam": lam0,
                   "c0_times_d": args.wc_c0d, "graph": "nsw", "degree": 16, "max_degree": 32,
                   "ef_construction": 256, "rho_runs": args.wc_rho_runs, "rho_queries": rho_q},
        "study": study,
        "recall_bound": rho,
    }
    print(json.dumps(out), flush=True)


def dynamic(args):
    """Insert(x) / Delete(x) of the dynamic setting (App. C) on the GPU path.

    An NSW index of the 1M x 128 mixture is built on its first 900,000
    points, takes the last 100,000 by Insert(x) in batches of 10,000, then
    loses 100,000 random points by Delete(x) in batches of 10,000.  Recall@10
    (FP32 rows, sampled queries) is measured after each phase and compared
    with a fresh build on the final point set."""
    import torch
    import paper_2505_17368_amd as hn
    import workloads as wl
    hn.load_library()
    dev = torch.device("cuda:0")
    X, Q = wl.make("gmm100_1M_d128")
    n, nq = X.shape[0], Q.shape[0]
    n0, batch, n_del = 900_000, 10_000, 100_000
    Xd, Qd = torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev)
    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(nq, min(args.gt_sample, nq), replace=False))
    bp = dict(degree=args.degree, max_degree=args.max_degree, graph=hn.GRAPH["nsw"],
              ef_construction=args.ef_construction, insert_shift=args.insert_shift,
              root_complete_max=args.root_max)
    efs = (64, 128, 192)

    def recall(idx, live, id_map=None):
        _, gt = exact_knn(X[live], Q[sample], 10, 0)
        out = {}
        for ef in efs:
            ids, _ = hn.henn_search_batch(idx, Qd, k=10, ef=ef)
            torch.cuda.synchronize()
            ids = ids.cpu().numpy()[sample]
            if id_map is not None:
                ids = np.where(ids >= 0, id_map[np.maximum(ids, 0)], -1)
            out[ef] = round(recall_at_k(ids, gt, X, Q[sample]), 4)
        return out

    torch.cuda.synchronize()
    t = time.time()
    idx = hn.henn_build(Xd[:n0].contiguous(), **bp)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"build on {n0} points: {build_s:.2f}s")
    t = time.time()
    for b in range(n0, n, batch):
        hn.henn_insert(idx, Xd[b:b + batch].contiguous())
    torch.cuda.synchronize()
    ins_s = time.time() - t
    rec_ins = recall(idx, np.arange(n))
    log(f"insert {n - n0} points in {ins_s:.2f}s ({(n - n0) / ins_s:,.0f}/s); recall {rec_ins}")
    gone = np.sort(rng.choice(n, n_del, replace=False)).astype(np.int32)
    t = time.time()
    for b in range(0, n_del, batch):
        hn.henn_delete(idx, gone[b:b + batch])
    torch.cuda.synchronize()
    del_s = time.time() - t
    live = np.setdiff1d(np.arange(n), gone)
    rec_del = recall(idx, live)
    layers = [idx.layer_info(i)["size"] for i in range(idx.num_layers)]
    log(f"delete {n_del} points in {del_s:.2f}s ({n_del / del_s:,.0f}/s); recall {rec_del}; "
        f"layers {layers}")
    idx.free()
    torch.cuda.synchronize()
    t = time.time()
    fresh = hn.henn_build(Xd[torch.from_numpy(live).to(dev)].contiguous(), **bp)
    torch.cuda.synchronize()
    fresh_s = time.time() - t
    rec_fresh = recall(fresh, live, id_map=live)
    log(f"fresh build on the final {len(live)} points: {fresh_s:.2f}s; recall {rec_fresh}")
    fresh.free()
    out = {
        "metric": "Insert(x) throughput into a 1M x 128 NSW index (batches of 10,000)",
        "value": round((n - n0) / ins_s, 1), "unit": "points/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gmm100_1M_d128", "n0": n0, "inserted": n - n0,
                   "deleted": n_del, "batch": batch, "graph": "nsw", "degree": args.degree,
                   "max_degree": args.max_degree, "ef_construction": args.ef_construction},
        "build_s": round(build_s, 2), "insert_s": round(ins_s, 2),
        "delete_points_per_s": round(n_del / del_s, 1), "delete_s": round(del_s, 2),
        "recall_after_insert": rec_ins, "recall_after_delete": rec_del,
        "fresh_build_s": round(fresh_s, 2), "recall_fresh_build": rec_fresh,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
