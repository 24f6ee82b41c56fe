#!/usr/bin/env python3
"""Search throughput on one MI355X: QPS at recall@10 >= 0.9, batched BF16
scan with FP32 rerank against the plain FP32 scan.

Workload (default `precision-10m-d768-bf16`): 10M x 768 unit-norm vectors
from a 1,000-component Gaussian mixture with Zipf(1.1) component weights (so
partition sizes follow a power law), stored FP32 with a BF16 copy, 4,096
k-means partitions, inner product, 16,384 queries per step (database rows
plus N(0, 0.1^2) noise, renormalised), k = 10, adaptive partition scanning
with f_M = 0.05.  The paper's datasets are not available; this seeded
mixture stands in for them.

`--workload two-level-50m-d128-f16`: 50M x 128 rows drawn around 50,000
generator-defined leaves (Zipf(1.1) leaf sizes), the leaves' centres as the
level-0 centroids (each row stored in its nearest), 64 top partitions over
them, L2, FP16 copy, 65,536 queries per step, f_M = 0.015 (750 level-0
candidates from the level-1 search at recall target 0.99 over 25% of the
top partitions).  The per-level split times the level-1 search with the
level-0 candidate geometry (quake_candidates) on its own.

Recall is measured against FP64 exact ground truth (the CPU oracle) on a
seeded 1,000-query subsample.  Both paths are run at recall targets 0.8,
0.9 and 0.95 (recall and the BF16 - FP32 gap reported per target); the
timed target of each path is the smallest of a ladder whose measured
recall@10 is >= 0.9.

One step = one search call over the whole batch: centroid scoring,
candidate selection and bisector geometry, the scan rounds (planning,
partition scans, in-order commit with the recall model), the FP32 rerank
(batched path) and the outputs.  Inputs are resident in HBM before the timed
region starts.

`value` is the batched BF16 path's QPS over the timed steps; the plain FP32
path is reported beside it (fewer steps: one of its steps takes about a
second).  Kernel durations come from a second pass over the same steps with
the library's HIP-event profiler on.  The batched path's scheduling knobs
(work-item size, grid, rounds between host checks, windows; never the
results) are autotuned on a separate seeded query batch; the plain path
keeps the defaults.

Roofline (`roofline`, the batched path's scan kernel k_scan_mfma):
achieved = algorithmic bytes per launch / HIP-event time per launch, where
the algorithmic bytes are every vector of every partition a scan round
touches, read once, x d x 2 bytes (BF16).  `traffic` is FETCH_SIZE +
WRITE_SIZE per launch from the committed rocprofv3 counter summary of this
workload when it was taken on the current kernel source and knobs, else
null.  The plain FP32 scan's roofline sits under `plain_fp32`: its
algorithmic bytes count every (query, vector) read (no reuse between
queries by design), most of which the caches serve, so its HBM fraction is
taken from the counters when they match.  The CPU oracle is timed on a
bounded sample of the same queries at the batched path's recall target.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC_NAME = "QPS at recall@10≥0.9, batched BF16 vs plain FP32 scan; scan HBM GB/s"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
REPORT_TARGETS = (0.8, 0.9, 0.95)
LADDER = (0.8, 0.9, 0.92, 0.94, 0.95, 0.96, 0.97, 0.98, 0.99, 1.0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def profiled_traffic(kernel, workload, source, knobs):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary profiles/<kernel>_<workload>.md, when it was taken with these
    knobs and the kernel's source file has not changed since; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    src = os.path.join(ROOT, "paper_2506_03437_amd", "csrc", source)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if " = " in line and not line.startswith(" "):
            k, v = line.rstrip("\n").split(" = ", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    # how many rounds are enqueued per host sync, and graph replay, leave the
    # scan launches themselves unchanged
    same = ("rounds_per_sync", "no_graph")
    want = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in fields.get("knobs", "").split(",") if "=" in kv}
    want = {k: v for k, v in want.items() if k not in same and v}
    have = {k: v for k, v in (knobs or {}).items() if v and k not in same}
    if fields.get("kernel_source_sha256") != sha or want != have or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def ground_truth(X, Qs, k, metric, threads):
    """Exact k-NN of the sample queries by the CPU oracle, over row blocks in
    parallel threads (BLAS single-threaded inside each), merged per query."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import knn as oknn

    n = X.shape[0]
    step = 262_144
    blocks = [(lo, min(n, lo + step)) for lo in range(0, n, step)]

    def work(b):
        lo, hi = b
        return oknn.knn_exact(X[lo:hi], np.arange(lo, hi, dtype=np.int64), Qs, k, metric,
                              query_block=Qs.shape[0])

    with threadpool_limits(limits=1):
        with ThreadPoolExecutor(max_workers=threads) as ex:
            parts = list(ex.map(work, blocks))
    ids, vals = parts[0]
    for pi, pv in parts[1:]:
        for j in range(Qs.shape[0]):
            ids[j], vals[j] = oknn.merge_topk(ids[j], vals[j], pi[j], pv[j], k, metric)
    return ids


def cpu_baseline_leg(X, Q, sample_rows, idx, workload, tau, seconds, gt_seconds, gt_threads):
    """The CPU oracle on the host: adaptive partition scanning over the
    device index's own partitioning at the GPU leg's recall target, timed on
    as many sample queries as fit in `seconds`."""
    import numpy as np
    from oracle import aps as oaps
    from oracle import ivf as oivf

    from oracle import twolevel as otl

    C, eids, epart = idx.export()
    C = C.cpu().numpy()
    assign = np.empty(X.shape[0], dtype=np.int64)
    assign[eids.cpu().numpy()] = epart.cpu().numpy()
    ps = oivf.PartitionedSet(X, np.arange(X.shape[0]), assign, C)
    table = oaps.CapTable(X.shape[1])
    if workload.leaves is not None:
        from paper_2506_03437_amd import quake_export_top
        C1, top_of = quake_export_top(idx.handle, X.shape[1], workload.nlist_top)
        tl = otl.TwoLevelSet(ps, top_of.cpu().numpy().astype(np.int64), C1.cpu().numpy())
        tparams = otl.TwoLevelParams(k=10, recall_target=tau, f_M=workload.f_M, metric=workload.metric)

        def one(q):
            otl.two_level_search_one(tl, q, tparams, table)
        what = "two-level adaptive partition scanning (level 1: target 0.99, f_M 0.25)"
    else:
        params = oaps.APSParams(k=10, recall_target=tau, f_M=workload.f_M, metric=workload.metric)

        def one(q):
            oaps.aps_search_one(ps, q, params, table)
        what = "adaptive partition scanning"
    Qs = Q[sample_rows]
    cores = len(os.sched_getaffinity(0))
    done = 0
    t0 = time.perf_counter()
    while done < Qs.shape[0] and time.perf_counter() - t0 < seconds:
        one(Qs[done])
        done += 1
    t_aps = time.perf_counter() - t0
    base = {
        "value": done / t_aps, "unit": "queries/s", "cores": cores, "kind": "oracle",
        "sample": (f"{done} of the workload's queries, FP64 NumPy {what} "
                   f"(recall target {tau}, the batched GPU leg's) over the device index's partitioning, "
                   f"{t_aps:.1f} s"),
    }
    if gt_seconds:
        base["brute_force"] = {
            "value": sample_rows.size / gt_seconds, "unit": "queries/s", "threads": gt_threads,
            "sample": f"exact FP64 k-NN of {sample_rows.size} queries over all {X.shape[0]} rows, "
                      f"{gt_seconds:.1f} s ({gt_threads} threads over row blocks, BLAS single-threaded each)"}
    return base


def serving_leg(make_index, w, X, tau, rates, n_requests, hbm_budget, rerank_factor, overlap, compare):
    """Continuous batching through the serving loop on the same index: a
    trace of single-query requests (Zipf(1.2) over the mixture components,
    popular set re-drawn every 10,000 requests) with a 1% insert batch and a
    1% delete batch after every 10,000 queries.  Each offered rate replays the
    trace open-loop with Poisson arrivals; the closed-loop run submits it all
    at once (the sustained rate).  Latency = arrival (enqueue) to answer ready.
    By default an update waits for the running searches to finish; with
    `overlap` it is applied beside the searches admitted before it (on a
    second copy of the store); `compare` adds a closed-loop run in the other
    mode.  Every run
    starts from a fresh build of the same index (make_index); the submitter
    sleeps between arrivals so that the library's allocator callbacks, which
    take the interpreter lock, are not held up by it."""
    import numpy as np
    import synth
    from paper_2506_03437_amd import Server

    n_live = X.shape[0]
    ts = synth.TraceSpec(n_requests=n_requests, drift_every=10_000, update_every=10_000, update_frac=0.01,
                         new_components=10)
    events = synth.serving_trace(w.spec, np.arange(n_live, dtype=np.int64), ts)
    kw = dict(k=w.k, recall_target=tau, f_M=w.f_M, scan_mode="batched", scan_dtype=w.storage,
              rerank_factor=rerank_factor)

    def replay(rate, overlapped=overlap):
        rng = np.random.default_rng(11)
        idx = make_index()
        with Server(idx, hbm_budget_bytes=hbm_budget, overlap_updates=overlapped, **kw) as srv:
            slots = srv.stats()["slots"]
            tickets, upd = [], []
            t0 = time.perf_counter()
            t_next = 0.0
            for ev in events:
                if ev[0] == "search":
                    Qb = ev[1]
                    if rate is None:
                        tickets += srv.search(Qb)
                        continue
                    arr = t_next + np.cumsum(rng.exponential(1.0 / rate, Qb.shape[0]))
                    t_next = float(arr[-1])
                    i = 0
                    while i < Qb.shape[0]:
                        now = time.perf_counter() - t0
                        j = int(np.searchsorted(arr, now, side="right"))
                        if j > i:
                            tickets += srv.search(Qb[i:j])
                            i = j
                        else:
                            time.sleep(max(0.0, min(float(arr[i]) - now, 1e-3)))
                elif ev[0] == "insert":
                    upd.append(srv.insert(ev[1], ev[2]))
                else:
                    upd.append(srv.delete(ev[1]))
            for t in tickets:
                srv.wait(t, 300.0)
            statuses = [srv.wait(t, 300.0)[3] for t in upd]
            st = srv.stats()
        idx.free()
        assert all(x == 0 for x in statuses), f"update batches failed: {statuses}"
        return {"offered_qps": rate, "achieved_qps": st["qps"], "p50_ms": st["p50_latency_s"] * 1e3,
                "p99_ms": st["p99_latency_s"] * 1e3, "mean_ms": st["mean_latency_s"] * 1e3,
                "completed": st["completed"], "slots": slots, "max_in_flight": st["max_in_flight"],
                "rounds": st["rounds"], "update_batches": len(statuses),
                "overlapped_updates": st["overlapped_updates"], "updates_beside_searches": overlapped}

    out = {"trace": f"{n_requests} single-query requests, Zipf(1.2) components drifting every 10,000, "
                    f"1% insert + 1% delete batch every 10,000 queries", "hbm_budget_bytes": hbm_budget,
           "recall_target": tau, "start": f"{n_live} rows of {w.name}", "updates_beside_searches": overlap,
           "runs": []}
    closed = replay(None)
    out["sustained"] = closed
    log(f"serving closed-loop: {closed['achieved_qps']:.0f} QPS, p50 {closed['p50_ms']:.2f} ms, "
        f"p99 {closed['p99_ms']:.2f} ms, slots {closed['slots']}, "
        f"{closed['overlapped_updates']} of {closed['update_batches']} updates beside running searches")
    if compare:
        other = replay(None, overlapped=not overlap)
        out["sustained_other_update_mode"] = other
        log(f"serving closed-loop, {'draining at' if overlap else 'beside'} updates: {other['achieved_qps']:.0f} QPS, "
            f"p50 {other['p50_ms']:.2f} ms, p99 {other['p99_ms']:.2f} ms")
    for r in rates:
        res = replay(r)
        out["runs"].append(res)
        log(f"serving at {r:.0f} QPS offered: {res['achieved_qps']:.0f} QPS, p50 {res['p50_ms']:.2f} ms, "
            f"p99 {res['p99_ms']:.2f} ms")
    return out


def maintenance_leg(idx, w, X, tau_r, rerank_factor, threads):
    """Adaptive maintenance (Sec. 4) after skewed growth: the serving trace's
    insert batches (new mixture components, 3 x 1% of the rows) go into the
    index, which piles them into the few partitions nearest to the new
    components; queries are half the trace's skewed searches (Zipf(1.2) over
    the components) and half new rows plus noise.  One batch fills the
    access counters, lambda(s) is profiled on this GPU for the batched path,
    one maintenance pass runs (alpha 0.9, r_f 50, one refinement pass,
    deletes below 64 vectors), and a second batch is timed and its recall
    measured before and after."""
    import numpy as np
    import torch
    import synth

    dev = torch.device("cuda", 0)
    n0 = X.shape[0]
    ts = synth.TraceSpec(n_requests=2 * w.nq, drift_every=10 ** 9, update_every=w.nq // 2, update_frac=0.01,
                         zipf_s=1.2)
    events = synth.serving_trace(w.spec, np.arange(n0, dtype=np.int64), ts)
    Qt = np.concatenate([e[1] for e in events if e[0] == "search"])
    ins = [e for e in events if e[0] == "insert"][:3]
    Xi = np.concatenate([e[1] for e in ins])
    ids_i = np.concatenate([e[2] for e in ins])
    sizes0 = idx.stats()
    idx.insert(torch.from_numpy(Xi).to(dev), torch.from_numpy(ids_i).to(dev))
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    half = w.nq // 2

    def batch(off):
        new = Xi[rng.choice(Xi.shape[0], half, replace=False)] + 0.1 * rng.standard_normal((half, X.shape[1]))
        new = (new / np.linalg.norm(new, axis=1, keepdims=True)).astype(np.float32)
        q = np.concatenate([Qt[off:off + w.nq - half], new])
        return np.ascontiguousarray(q[rng.permutation(q.shape[0])])

    QA = torch.from_numpy(batch(0)).to(dev)
    QB_h = batch(w.nq)
    QB = torch.from_numpy(QB_h).to(dev)
    sample = np.sort(rng.choice(w.nq, 300, replace=False))
    # ground truth over the grown set: ids of the new rows follow the old ones
    truth = ground_truth(np.concatenate([X, Xi]), QB_h[sample], 10, w.metric, threads)
    row_id = np.concatenate([np.arange(n0, dtype=np.int64), ids_i])
    truth = row_id[truth]
    kw = dict(k=w.k, recall_target=tau_r, f_M=w.f_M, scan_mode="batched", scan_dtype=w.storage,
              rerank_factor=rerank_factor)

    def timed():
        idx.search(QB, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ids, _, ns, _ = idx.search(QB, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 5
        found = ids.cpu().numpy()[sample]
        rec = float(np.mean([len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(sample.size)])) / 10
        return {"ms_per_search": ms, "qps": w.nq / ms * 1e3, "recall_at_10": rec,
                "mean_partitions_scanned": float(ns.float().mean().item()), "nlist": idx.stats()[1]}

    before = timed()
    log(f"maintenance: after {Xi.shape[0]} skewed inserts: {before['qps']:.0f} QPS, recall {before['recall_at_10']:.4f}")
    sizes = [64, 256, 1024, 4096, 16384, 65536]
    lam = idx.profile_latency(sizes, nq=4096, reps=3, **kw)
    idx.access_stats(reset=True)
    idx.search(QA, **kw)
    torch.cuda.synchronize()
    hits, window = idx.access_stats()
    # the paper's threshold is 250 ns against millisecond queries; here a
    # query costs about a microsecond of a batch, so the same ratio (1e-4)
    tau = 1e-4 * before["ms_per_search"] * 1e3 / w.nq
    t0 = time.perf_counter()
    rep, dec = idx.maintain(sizes, lam, tau=tau, alpha=0.9, refine_radius=50, refine_iters=1, merge_below=64)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    after = timed()
    log(f"maintenance: {rep['splits']} splits, {rep['deletes']} deletes in {t_m:.1f} s; after: "
        f"{after['qps']:.0f} QPS, recall {after['recall_at_10']:.4f}")
    return {"setup": f"{Xi.shape[0]} rows inserted from new mixture components into {sizes0[0]} rows; queries per "
                     f"batch: half Zipf(1.2) over the components, half new rows plus N(0, 0.1^2) noise; "
                     f"statistics from one batch, timing and recall on a second",
            "lambda_sizes": sizes, "lambda_us_per_query": lam.tolist(), "tau_us": tau, "window": int(window),
            "partitions_hit": int((hits > 0).sum()), "report": rep, "seconds": t_m, "before": before,
            "after": after, "decisions_committed": int(sum(1 for d in dec if d["committed"]))}


def min_nprobe_per_query(key, part_of, truth, need):
    """For each query (row of `key`, its centroid keys, smaller is nearer;
    ties by partition number), the fewest nearest partitions that together
    hold `need` of its true neighbours (`truth` rows, `part_of` maps a row to
    its partition)."""
    import numpy as np
    rank = np.empty(key.shape, dtype=np.int64)
    rank[np.arange(key.shape[0])[:, None], np.argsort(key, axis=1, kind="stable")] = np.arange(key.shape[1])[None, :]
    nb_rank = np.sort(np.take_along_axis(rank, part_of[truth], axis=1), axis=1)
    return nb_rank[:, need - 1] + 1


def ablation_leg(idx, w, Q, Qd, truth, sample_rows, recall_of, paths, upper):
    """Estimator and early-termination ablations on synthetic data.

    * Estimators (Sec. 5.1, Table tab:recall_overhead): APS (recompute when
      rho moved by more than 1%, table), APS-R (recompute after every
      partition, table) and APS-RP (every partition, incomplete beta on the
      device) at recall target 0.9 on each path: recall@10, partitions
      scanned, time per search and the commit kernel's time (where the
      estimator runs).
    * Early termination (Sec. 7, Table tab:early_term) at targets 0.8, 0.9
      and 0.99 on the first path: APS; a fixed nprobe tuned by binary search
      over the ground-truth sample (the tuning time is reported); and the
      per-query oracle, the fewest nearest partitions that hold ceil(target k)
      of the query's true neighbours (a lower bound on partitions; its time
      groups the sample queries by their nprobe, one search per group).
    * f_M (Sec. 8, "Setting System Parameters"): 0.01 to 0.1 at target 0.9.
    """
    import math
    import numpy as np
    import torch

    def sync():
        torch.cuda.synchronize()

    def timed(Qx, steps=5, **kw):
        idx.search(Qx, k=w.k, **upper, **kw)
        sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = idx.search(Qx, k=w.k, **upper, **kw)
        sync()
        return out, (time.perf_counter() - t0) * 1e3 / steps

    def commit_ms(**kw):
        idx.profile(enable=True, reset=True)
        sync()
        idx.search(Qd, k=w.k, **upper, **kw)
        sync()
        prof = idx.profile(enable=False, reset=True)
        return prof["commit"][1], sum(v[1] for k, v in prof.items() if k != "scan_sets")

    res = {"estimators": {}, "early_termination": {}, "f_M": {}}
    for p, pkw in paths.items():
        rows = []
        base_ns = None
        for est in ("aps", "aps-r", "aps-rp"):
            (ids, _, ns, rec), ms = timed(Qd, recall_target=0.9, f_M=w.f_M, estimator=est, **pkw)
            cms, kms = commit_ms(recall_target=0.9, f_M=w.f_M, estimator=est, **pkw)
            nsn = ns.cpu().numpy()
            base_ns = nsn if base_ns is None else base_ns
            rows.append({"estimator": est, "recall_at_10": recall_of(ids), "ms_per_search": ms,
                         "commit_ms_per_search": cms, "kernel_ms_per_search": kms,
                         "mean_partitions_scanned": float(nsn.mean()),
                         "mean_recall_estimate": float(rec.double().mean().item()),
                         "same_stop_as_aps": float((nsn == base_ns).mean())})
            log(f"ablation {p} {est}: recall {rows[-1]['recall_at_10']:.4f}, {ms:.2f} ms per search, "
                f"commit {cms:.3f} ms, partitions {rows[-1]['mean_partitions_scanned']:.2f}")
        res["estimators"][p] = rows

    p0 = next(iter(paths))
    pkw = paths[p0]
    Qs = Qd[torch.from_numpy(sample_rows).to(Qd.device)]
    # the per-query oracle: partition ranks of each query's true neighbours
    C, eids, epart = idx.export()
    C = C.cpu().numpy().astype(np.float64)
    part_of = np.empty(int(eids.max().item()) + 1, dtype=np.int64)
    part_of[eids.cpu().numpy()] = epart.cpu().numpy()
    Qh = Q[sample_rows].astype(np.float64)
    if w.metric == "ip":
        key = -(Qh @ C.T)
    else:
        key = (Qh * Qh).sum(1)[:, None] - 2.0 * Qh @ C.T + (C * C).sum(1)[None, :]
    nlist = C.shape[0]
    limit = min(nlist, 4096)
    for tau in (0.8, 0.9, 0.99):
        need = int(math.ceil(tau * w.k - 1e-9))
        row = {}
        (ids, _, ns, _), ms = timed(Qd, recall_target=tau, f_M=w.f_M, **pkw)
        (sids, _, sns, _), sms = timed(Qs, recall_target=tau, f_M=w.f_M, **pkw)
        row["aps"] = {"recall_at_10": recall_of(ids), "ms_per_search": ms,
                      "mean_partitions_scanned": float(ns.float().mean().item()),
                      "sample_mean_partitions_scanned": float(sns.float().mean().item()),
                      "sample_ms_per_search": sms}
        # fixed nprobe: the smallest whose mean recall over the sample reaches tau
        t0 = time.perf_counter()
        lo, hi, probes = 1, limit, 0
        while lo < hi:
            mid = (lo + hi) // 2
            fids, _, _, _ = idx.search(Qs, k=w.k, nprobe=mid, **upper, **pkw)
            found = fids.cpu().numpy()
            probes += 1
            r = float(np.mean([len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(found.shape[0])]))
            if r / w.k >= tau:
                hi = mid
            else:
                lo = mid + 1
        tune_s = time.perf_counter() - t0
        (fids, _, _, _), fms = timed(Qd, nprobe=lo, **pkw)
        (_, _, _, _), fsms = timed(Qs, nprobe=lo, **pkw)
        row["fixed"] = {"nprobe": lo, "tuning_seconds": tune_s, "tuning_searches": probes,
                        "recall_at_10": recall_of(fids), "ms_per_search": fms, "sample_ms_per_search": fsms}
        # APS at the smallest target of the ladder whose measured recall reaches tau
        for t in LADDER:
            (mids, _, mns, _), mms = timed(Qd, recall_target=t, f_M=w.f_M, **pkw)
            if recall_of(mids) >= tau or t == LADDER[-1]:
                break
        row["aps_matched"] = {"recall_target": t, "recall_at_10": recall_of(mids), "ms_per_search": mms,
                              "mean_partitions_scanned": float(mns.float().mean().item())}
        # the per-query oracle
        onp = min_nprobe_per_query(key, part_of, truth, need)
        t_or = 0.0
        found = np.empty((sample_rows.size, w.k), dtype=np.int64)
        groups = np.unique(onp)
        for v in groups.tolist():
            sel = np.nonzero(onp == v)[0]
            Qg = Qs[torch.from_numpy(sel).to(Qd.device)]
            idx.search(Qg, k=w.k, nprobe=int(v), **upper, **pkw)
            sync()
            t0 = time.perf_counter()
            gids, _, _, _ = idx.search(Qg, k=w.k, nprobe=int(v), **upper, **pkw)
            sync()
            t_or += time.perf_counter() - t0
            found[sel] = gids.cpu().numpy()
        orec = float(np.mean([len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(found.shape[0])]))
        row["oracle"] = {"mean_partitions_scanned": float(onp.mean()), "recall_at_10": orec / w.k,
                         "sample_ms_grouped": t_or * 1e3, "groups": int(groups.size)}
        log(f"ablation {p0} target {tau}: APS recall {row['aps']['recall_at_10']:.4f} over "
            f"{row['aps']['mean_partitions_scanned']:.1f} partitions; fixed nprobe {lo} ({tune_s:.1f} s tuning) recall "
            f"{row['fixed']['recall_at_10']:.4f}; oracle {row['oracle']['mean_partitions_scanned']:.1f} partitions")
        res["early_termination"][str(tau)] = row

    for p, pkw in paths.items():
        rows = []
        for f in (0.01, 0.02, 0.05, 0.1):
            (ids, _, ns, _), ms = timed(Qd, recall_target=0.9, f_M=f, **pkw)
            rows.append({"f_M": f, "candidates": int(math.ceil(f * nlist - 1e-9)), "recall_at_10": recall_of(ids),
                         "ms_per_search": ms, "mean_partitions_scanned": float(ns.float().mean().item())})
            log(f"ablation {p} f_M {f}: recall {rows[-1]['recall_at_10']:.4f}, {ms:.2f} ms, "
                f"partitions {rows[-1]['mean_partitions_scanned']:.2f}")
        res["f_M"][p] = rows
    return res


def levels_leg(idx, w, Qd, recall_of, path_kw):
    """One, two and three levels over the same level 0 (Sec. 3; Sec. 4.2
    "Add Level"; Sec. 7 "Multi-Level Recall Estimation", Table
    tab:two_level_results): a level of round(sqrt(N)) partitions is added on
    top of the current one twice, and each configuration is searched at
    level-0 targets 0.8 / 0.9 / 0.95 with the upper levels at 0.99 over 25%
    of their partitions.  The upper-level time is the candidate search
    alone (quake_candidates, which runs the upper levels and the level-0
    geometry); the levels are removed afterwards."""
    import math
    import torch

    def timed(fn, steps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / steps

    res = []
    added = 0
    for levels in (1, 2, 3):
        if levels > 1:
            top = idx.level_sizes()[levels - 2]
            idx.add_level(max(1, int(round(math.sqrt(top)))), kmeans_iters=10, seed=levels)
            added += 1
        up = dict(upper_recall_target=0.99, upper_f_M=0.25) if levels > 1 else {}
        sizes = idx.level_sizes()
        for tau in (0.8, 0.9, 0.95):
            (ids, _, ns, _), ms = timed(lambda: idx.search(Qd, k=w.k, recall_target=tau, f_M=w.f_M, **up, **path_kw))
            _, cms = timed(lambda: idx.candidates(Qd, w.f_M, **up))
            row = {"levels": levels, "partitions_per_level": sizes[:levels], "recall_target": tau,
                   "recall_at_10": recall_of(ids), "ms_per_search": ms, "candidates_ms": cms,
                   "mean_partitions_scanned": float(ns.float().mean().item())}
            res.append(row)
            log(f"levels {levels} {sizes[:levels]} target {tau}: recall {row['recall_at_10']:.4f}, {ms:.2f} ms "
                f"(candidates {cms:.2f} ms), {row['mean_partitions_scanned']:.1f} partitions")
    for _ in range(added):
        idx.remove_level()
    return res


def filter_leg(w, sample_rows, threads):
    """Filtered search (Sec. 8, "Filters") on the workload's rows with
    seeded labels: one of 8 labels per row, the row's mixture component's
    home label with probability 0.7, else uniform; every query filters on
    one uniformly drawn label (about 1 row in 8 passes).  A labelled index of
    the same shape is built; recall@10 is against the exact filtered k-NN of
    the sample queries.  Reported: the filtered adaptive search at targets
    0.8 / 0.9 / 0.95 (plain FP32 path), a fixed nprobe tuned by binary search
    to filtered recall 0.9, and post-filtering (an unfiltered adaptive search
    for k / (pass rate) results, of which the first k passing are kept)."""
    import numpy as np
    import torch
    import synth
    from oracle import knn as oknn
    from paper_2506_03437_amd import Index

    dev = torch.device("cuda", 0)
    X, comp = synth.database(w.spec, with_components=True, threads=threads)
    Q = synth.queries(w.spec, w.nq, noise_std=w.query_noise, threads=threads)
    attrs = synth.row_labels(w.spec, comp)
    masks = synth.query_masks(w.spec, w.nq)
    as_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    idx = Index(Xd, metric=w.metric, nlist=w.nlist, kmeans_iters=10, seed=1, attrs=as_dev(attrs))
    del Xd
    Qd = torch.from_numpy(Q).to(dev)
    Md = as_dev(masks)
    truth = np.empty((sample_rows.size, w.k), dtype=np.int64)
    for lab in np.unique(masks[sample_rows]).tolist():
        sel = np.nonzero(masks[sample_rows] == lab)[0]
        rows = np.nonzero(attrs == lab)[0]
        ti, _ = oknn.knn_exact(X[rows], rows.astype(np.int64), Q[sample_rows[sel]], w.k, w.metric)
        truth[sel] = ti
    pass_rate = float(np.mean([(attrs == m).mean() for m in np.unique(masks)]))

    def recall(ids):
        found = ids[sample_rows] if ids.shape[0] == w.nq else ids
        return float(np.mean([len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(truth.shape[0])])) / w.k

    def timed(**kw):
        idx.search(Qd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            out = idx.search(Qd, **kw)
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / 3

    res = {"setup": "8 labels, home label of the row's component with probability 0.7; one label per query; "
                    f"mean pass rate {pass_rate:.3f}", "aps": []}
    for tau in (0.8, 0.9, 0.95):
        (ids, _, ns, _), ms = timed(k=w.k, recall_target=tau, f_M=w.f_M, filter=Md)
        res["aps"].append({"recall_target": tau, "recall_at_10": recall(ids.cpu().numpy()), "ms_per_search": ms,
                           "mean_partitions_scanned": float(ns.float().mean().item())})
        log(f"filters: APS target {tau}: recall {res['aps'][-1]['recall_at_10']:.4f}, "
            f"{res['aps'][-1]['mean_partitions_scanned']:.1f} partitions, {ms:.2f} ms")
    for t in LADDER:
        (ids, _, ns, _), ms = timed(k=w.k, recall_target=t, f_M=w.f_M, filter=Md)
        r = recall(ids.cpu().numpy())
        if r >= 0.9 or t == LADDER[-1]:
            break
    res["aps_matched"] = {"recall_target": t, "recall_at_10": r, "ms_per_search": ms,
                          "mean_partitions_scanned": float(ns.float().mean().item())}
    Qs = Qd[torch.from_numpy(sample_rows).to(dev)]
    Ms = Md[torch.from_numpy(sample_rows).to(dev)]
    lo, hi = 1, min(w.nlist, 4096)
    while lo < hi:
        mid = (lo + hi) // 2
        fids, _, _, _ = idx.search(Qs, k=w.k, nprobe=mid, filter=Ms)
        if recall(fids.cpu().numpy()) >= 0.9:
            hi = mid
        else:
            lo = mid + 1
    (fids, _, _, _), fms = timed(k=w.k, nprobe=lo, filter=Md)
    res["fixed_nprobe"] = {"nprobe": lo, "recall_at_10": recall(fids.cpu().numpy()), "ms_per_search": fms}
    kp = int(min(256, round(w.k / pass_rate)))
    (pids, _, pns, _), pms = timed(k=kp, recall_target=0.9, f_M=w.f_M)
    pids = pids.cpu().numpy()
    kept = np.full((w.nq, w.k), -1, dtype=np.int64)
    for i in sample_rows.tolist():
        ok = [j for j in pids[i].tolist() if j >= 0 and attrs[j] & masks[i]][: w.k]
        kept[i, : len(ok)] = ok
    res["post_filter"] = {"k_searched": kp, "recall_target": 0.9, "recall_at_10": recall(kept),
                          "ms_per_search": pms, "mean_partitions_scanned": float(pns.float().mean().item())}
    log(f"filters: APS target {t}: recall {r:.4f}; fixed nprobe {lo} recall {res['fixed_nprobe']['recall_at_10']:.4f} {fms:.2f} ms; post-filter "
        f"k={kp}: recall {res['post_filter']['recall_at_10']:.4f}, {pms:.2f} ms")
    idx.free()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3, help="timed steps of the plain FP32 path (at most --steps)")
    ap.add_argument("--workload", default="precision-10m-d768-bf16")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--recall-sample", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ground-truth", action="store_true", help="skip recall measurement (profiling runs)")
    ap.add_argument("--recall-target", type=float, default=0.0,
                    help="skip the ladder and time the paths at this target")
    ap.add_argument("--plain-recall-target", type=float, default=0.0,
                    help="with --recall-target: the plain path's own target (default: the same)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default scheduling knobs")
    ap.add_argument("--tuning", default="", help="knobs to set instead of autotuning, e.g. chunk_tiles=64,max_window=16")
    ap.add_argument("--tuning-path", default="batched", help="path (plain/batched) the --tuning knobs apply to")
    ap.add_argument("--paths", default="plain_fp32,batched_bf16",
                    help="comma list of plain_fp32, batched_<storage> and plain_pq8 (needs --pq-m)")
    ap.add_argument("--pq-m", type=int, default=0,
                    help="also keep product codes of this many subspaces (Sec. 8, vector compression): the "
                         "plain_pq8 path scans them and reranks --rerank-factor x k candidates in FP32")
    ap.add_argument("--rerank-factor", type=int, default=6,
                    help="batched path: FP32 rerank of this many x k candidates (6: the BF16 - FP32 recall@10 gap "
                         "stays within 0.005 on this workload; 4 loses about 0.01)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy a BYTES-long device buffer 5 times (calibrates HBM byte counters) and exit")
    ap.add_argument("--serving-requests", type=int, default=0, help="> 0 runs the serving-loop leg")
    ap.add_argument("--levels", action="store_true",
                    help="one, two and three levels over the workload's index (after the timed legs)")
    ap.add_argument("--ablation", action="store_true",
                    help="estimator, early-termination and f_M ablations on the workload (after the timed legs)")
    ap.add_argument("--maintenance", action="store_true",
                    help="run a maintenance pass under skewed queries and time them before and after")
    ap.add_argument("--serving-rates", default="20000,100000,400000")
    ap.add_argument("--serving-hbm-budget", type=int, default=256 << 20)
    ap.add_argument("--serving-overlap", action="store_true",
                    help="serving: apply each update beside the searches admitted before it (second store copy) "
                         "instead of draining them first")
    ap.add_argument("--serving-compare", action="store_true",
                    help="serving: add a closed-loop run in the other update mode")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the index is searched on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        dev = torch.device("cuda", 0)
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 5}), flush=True)
        return

    import synth
    from paper_2506_03437_amd import Index

    w = synth.get_workload(args.workload)
    two_level = w.leaves is not None
    threads = host_threads()
    t0 = time.perf_counter()
    if two_level:
        centres, _, X = synth.leaf_spec_database(w.leaves, threads=threads)
        Q = synth.leaf_spec_queries(w.leaves, X, w.nq, w.query_noise)
        Qtune_h = synth.leaf_spec_queries(w.leaves, X, w.nq, w.query_noise, stream_chunk=1)
    else:
        X = synth.database(w.spec, threads=threads)
        Q = synth.queries(w.spec, w.nq, noise_std=w.query_noise, threads=threads)
        Qtune_h = synth.queries(w.spec, w.nq, noise_std=w.query_noise, stream_chunk=1, threads=threads)
    log(f"generated {X.shape} database and {Q.shape} queries in {time.perf_counter() - t0:.1f} s "
        f"({threads} threads)")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    Xd = torch.from_numpy(X).to(dev)
    if two_level:
        # level 0: the generator's leaf centres (each row goes to its nearest);
        # level 1: k-means of those centres into nlist_top partitions
        idx = Index(Xd, metric=w.metric, nlist=w.nlist, storage=w.storage, n_levels=2, nlist_top=w.nlist_top,
                    centroids=torch.from_numpy(centres).to(dev), kmeans_iters=10, seed=1)
    else:
        # serving inserts: 5% spare capacity per partition and in the arena;
        # without the plain FP32 path the index keeps no FP32 tile copy
        idx = Index(Xd, metric=w.metric, nlist=w.nlist, storage=w.storage, kmeans_iters=10, seed=1,
                    capacity_slack=0.05 if args.serving_requests > 0 else 0.0,
                    f32_tiles="plain_fp32" in args.paths.split(","), pq_m=args.pq_m)
    del Xd
    torch.cuda.synchronize()
    log(f"built {w.nlist} partitions{f' under {w.nlist_top}' if two_level else ''} in "
        f"{time.perf_counter() - t0:.1f} s ({idx.stats()[2] / 1e9:.1f} GB of index memory)")
    Qd = torch.from_numpy(Q).to(dev)
    Qtune = torch.from_numpy(Qtune_h).to(dev)
    del Qtune_h
    # the upper level of a two-level index: recall target 0.99 over 25% of its partitions
    upper = dict(upper_recall_target=0.99, upper_f_M=0.25) if two_level else {}
    rng = np.random.default_rng(7)
    sample_rows = np.sort(rng.choice(w.nq, size=min(args.recall_sample, w.nq), replace=False))

    truth = None
    gt_seconds = 0.0
    if not args.no_ground_truth:
        t0 = time.perf_counter()
        truth = ground_truth(X, Q[sample_rows], 10, w.metric, threads)
        gt_seconds = time.perf_counter() - t0
        log(f"oracle exact k-NN for {sample_rows.size} queries: {gt_seconds:.1f} s")

    bkey = f"batched_{w.storage}"
    all_paths = {
        "plain_fp32": dict(scan_mode="plain", scan_dtype="f32"),
        bkey: dict(scan_mode="batched", scan_dtype=w.storage, rerank_factor=args.rerank_factor),
        "plain_pq8": dict(scan_mode="plain", scan_dtype="pq8", rerank_factor=args.rerank_factor),
    }
    paths = {(bkey if p.startswith("batched") else p): None for p in args.paths.split(",") if p}
    paths = {p: all_paths[p] for p in paths}

    def run(path, tau):
        return idx.search(Qd, k=w.k, recall_target=tau, f_M=w.f_M, **upper, **paths[path])

    def recall_of(ids):
        found = ids.cpu().numpy()[sample_rows]
        hits = [len(set(found[i].tolist()) & set(truth[i].tolist())) for i in range(found.shape[0])]
        return float(np.mean(hits)) / w.k

    # recall at the reported targets, and each path's smallest target of the
    # ladder reaching recall@10 >= 0.9
    ladder = {p: [] for p in paths}
    chosen = {}
    if truth is not None and not args.recall_target:
        for tau in LADDER:
            for p in paths:
                if p in chosen and tau not in REPORT_TARGETS:
                    continue
                ids, _, ns, _ = run(p, tau)
                torch.cuda.synchronize()
                rec = recall_of(ids)
                ladder[p].append({"recall_target": tau, "recall_at_10": rec,
                                  "mean_partitions_scanned": float(ns.float().mean().item())})
                log(f"{p}: recall target {tau}: recall@10 {rec:.4f}, mean partitions "
                    f"{ladder[p][-1]['mean_partitions_scanned']:.2f}")
                if rec >= 0.9 and p not in chosen:
                    chosen[p] = tau
            if all(p in chosen for p in paths) and tau >= max(REPORT_TARGETS):
                break
    for p in paths:
        fixed = args.plain_recall_target if p.startswith("plain") and args.plain_recall_target else args.recall_target
        chosen.setdefault(p, fixed or 0.95)

    def measure(path, steps):
        tau = chosen[path]
        knobs = None
        if args.tuning and path.startswith(args.tuning_path):
            # fixed knobs (to profile the configuration a tuned run chose)
            knobs = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tuning.split(",") if kv}
            idx.set_tuning(**knobs)
            log(f"{path}: knobs set to {knobs}")
        elif args.tuning or args.no_autotune or path.startswith("plain"):
            idx.set_tuning()
        else:
            # scheduling knobs (never the results) tuned on a separate seeded batch
            knobs, tuned_ms = idx.autotune(Qtune, reps=2, k=w.k, recall_target=tau, f_M=w.f_M, **upper,
                                           **paths[path])
            log(f"{path}: autotuned {knobs} ({tuned_ms:.2f} ms per search on the tuning batch)")
        for _ in range(min(args.warmup, 1) if path.startswith("plain") else args.warmup):
            run(path, tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = run(path, tau)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # kernel durations: the same steps again with the library's HIP-event
        # profiler on (it times each kernel class on the search stream, so the
        # rounds launch one by one instead of replaying captured graphs)
        idx.profile(enable=True, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run(path, tau)
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - t0
        prof = idx.profile(enable=False, reset=True)
        level_split = None
        if two_level:
            # the level-1 search and the level-0 candidate geometry alone (what
            # quake_candidates runs), timed over the same steps; level 0's
            # scan rounds and rerank are the rest of a step
            for _ in range(steps):
                idx.candidates(Qd, w.f_M, **upper)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                idx.candidates(Qd, w.f_M, **upper)
            torch.cuda.synchronize()
            up_ms = (time.perf_counter() - t0) * 1e3 / steps
            level_split = {"level1_and_candidates_ms": up_ms, "level0_ms": elapsed * 1e3 / steps - up_ms}
        ids, _, ns, _ = out
        rec = recall_of(ids) if truth is not None else None
        launches, ms, nbytes, flops = prof["scan"]
        res = {
            "qps": steps * w.nq / elapsed,
            "steps": steps,
            "ms_per_step": elapsed * 1e3 / steps,
            "ms_per_step_profiled": elapsed_prof * 1e3 / steps,
            "recall_target": tau,
            "recall_at_10": rec,
            "mean_partitions_scanned": float(ns.float().mean().item()),
            "scan_launches_per_step": launches / steps,
            "scan_ms_per_launch": ms / max(launches, 1),
            "scan_algorithmic_gbs": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0,
            "scan_tflops": flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0,
            "scan_bytes_per_launch": nbytes / max(launches, 1),
            "scan_flops_per_launch": flops / max(launches, 1),
            "kernels_ms_per_step": {k: v[1] / steps for k, v in prof.items() if v[0]},
            "tuning": knobs,
        }
        if level_split:
            res["per_level_ms_per_step"] = level_split
        if path.startswith("batched"):
            res["scan_set_bytes_per_launch"] = prof["scan_sets"][2] / max(launches, 1)
            res["scan_bytes_per_step"] = nbytes / steps
        non_scan = sum(v for k, v in res["kernels_ms_per_step"].items() if k != "scan")
        res["non_scan_share_of_kernel_time"] = non_scan / max(sum(res["kernels_ms_per_step"].values()), 1e-12)
        log(f"{path}: {res['qps']:.0f} QPS, {res['ms_per_step']:.2f} ms/step "
            f"({res['ms_per_step_profiled']:.2f} profiled), recall {rec}, "
            f"scan {res['scan_ms_per_launch']:.3f} ms x {res['scan_launches_per_step']:.1f} per step")
        return res

    results = {}
    for p in paths:
        results[p] = measure(p, min(args.plain_steps, args.steps) if p.startswith("plain") else args.steps)
    batched = results.get(bkey)
    plain = results.get("plain_fp32")

    cpu = None
    if not args.no_cpu_baseline and truth is not None:
        cpu = cpu_baseline_leg(X, Q, sample_rows, idx, w, chosen.get(bkey, chosen[next(iter(paths))]),
                               args.cpu_seconds, gt_seconds, threads)
    ablation = None
    if args.ablation and truth is not None:
        ablation = ablation_leg(idx, w, Q, Qd, truth, sample_rows, recall_of, paths, upper)
        if not two_level:
            ablation["filters"] = filter_leg(w, sample_rows, threads)
    levels = None
    if args.levels and truth is not None and not two_level:
        levels = levels_leg(idx, w, Qd, recall_of, paths[next(iter(paths))])
    maint = None
    if args.maintenance and batched is not None and not two_level:
        maint = maintenance_leg(idx, w, X, batched["recall_target"], args.rerank_factor, threads)
    serving = None
    if args.serving_requests > 0 and batched is not None:
        rates = [float(r) for r in args.serving_rates.split(",") if r]
        idx.free()
        idx = None

        def make_index():
            Xd = torch.from_numpy(X).to(dev)
            out = Index(Xd, metric=w.metric, nlist=w.nlist, storage=w.storage, kmeans_iters=10, seed=1,
                        capacity_slack=0.05, f32_tiles=False)
            del Xd
            if batched.get("tuning"):
                out.set_tuning(**batched["tuning"])  # the knobs the batched leg was timed with
            torch.cuda.synchronize()
            return out

        serving = serving_leg(make_index, w, X, batched["recall_target"], rates, args.serving_requests,
                              args.serving_hbm_budget, args.rerank_factor, args.serving_overlap,
                              args.serving_compare)

    pq = results.get("plain_pq8")
    if pq is not None:
        # algorithmic bytes: every (query, row) pair's codes and residual term;
        # the per-query code tables are gathered through L1 / L2 besides
        pq["roofline"] = {"bound": "hbm", "kernel": "k_scan_pq", "achieved": pq["scan_algorithmic_gbs"],
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": pq["scan_algorithmic_gbs"] / HBM_PEAK_GBS,
                          "traffic": None}
    roof = None
    if batched is not None:
        ms = batched["scan_ms_per_launch"]
        gbs = batched["scan_algorithmic_gbs"]
        tfl = batched["scan_tflops"]
        traffic = profiled_traffic("k_scan_mfma", w.name, "k_batched.hip", batched["tuning"])
        roof = {"bound": "hbm", "kernel": "k_scan_mfma", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_gbs": traffic / (ms * 1e-3) / 1e9 if traffic and ms > 0 else None,
                "algorithmic_bytes_per_launch": batched["scan_bytes_per_launch"],
                "set_bytes_per_launch": batched["scan_set_bytes_per_launch"],
                "ms_per_launch": ms, "mfma_tflops": tfl, "mfma_frac": tfl / MFMA_BF16_PEAK_TFLOPS,
                "flops_per_launch": batched["scan_flops_per_launch"]}
        if roof["mfma_frac"] > roof["frac"]:
            roof.update({"bound": "mfma", "achieved": tfl, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": roof["mfma_frac"]})
    if plain is not None:
        ms = plain["scan_ms_per_launch"]
        traffic = profiled_traffic("k_scan_f32", w.name, "k_scan.hip", None)
        hbm = traffic / (ms * 1e-3) / 1e9 if traffic and ms > 0 else None
        plain["roofline"] = {"bound": "hbm", "kernel": "k_scan_f32", "achieved": hbm, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS if hbm else None, "traffic": traffic,
                             "algorithmic_gbs": plain["scan_algorithmic_gbs"],
                             "algorithmic_note": "every (query, vector) read counted; caches serve most re-reads"}
    gap = []
    if "plain_fp32" in ladder and bkey in ladder:
        for tau in REPORT_TARGETS:
            a = [e for e in ladder["plain_fp32"] if e["recall_target"] == tau]
            b = [e for e in ladder[bkey] if e["recall_target"] == tau]
            if a and b:
                gap.append({"recall_target": tau, "fp32": a[0]["recall_at_10"],
                            f"{w.storage}_rerank": b[0]["recall_at_10"],
                            "gap": b[0]["recall_at_10"] - a[0]["recall_at_10"]})
    head = batched or plain or next(iter(results.values()))
    line = {
        "metric": METRIC_NAME,
        "value": head["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.storage if batched else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.spec.n, "d": w.spec.d, "nlist": w.nlist, "metric": w.metric,
                   "queries_per_step": w.nq, "k": w.k, "recall_target": head["recall_target"], "f_M": w.f_M,
                   "path": f"batched {w.storage.upper()} MFMA scan + FP32 rerank of {args.rerank_factor}k "
                           "candidates, adaptive partition scanning"
                           + (f"; two levels ({w.nlist_top} top partitions, level-1 target 0.99 over 25%)"
                              if two_level else "")},
        "recall_at_10": head["recall_at_10"],
        "speedup_vs_plain_fp32": batched["qps"] / plain["qps"] if batched and plain else None,
        "roofline": roof,
        "recall_by_target": ladder,
        f"recall_gap_{w.storage}_minus_fp32": gap,
        bkey: batched,
        "plain_fp32": plain,
        "plain_pq8": results.get("plain_pq8"),
        "serving": serving,
        "maintenance": maint,
        "ablation": ablation,
        "levels": levels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if idx is not None:
        idx.free()


if __name__ == "__main__":
    main()
