"""Adaptive maintenance on the device against the maintenance oracle (Sec. 4).

* Access counters (Stage 0 of the decision workflow): with fixed nprobe a
  query scans exactly its nprobe nearest partitions, so the device's counts
  must equal the oracle's FP64 centroid ranking (up to near-ties at the
  nprobe-th place); with adaptive scanning every search adds exactly the
  partitions it committed (sum of hits = sum of partitions scanned), and
  the counts follow the oracle's replay of each query except queries whose
  stop decision falls within the margin.
* A maintenance pass over an index whose partitions are pairs of separated
  groups (so that every 2-means split and every nearest-centroid step is
  far from a tie): hot balanced pairs are split and committed, hot
  unbalanced pairs are split tentatively and rejected at the verify step,
  cold pairs are left alone, tiny unvisited partitions next to cold pairs
  are deleted.  The decisions (with their estimated and verified deltas),
  the final partition of every vector and the centroids must equal the
  oracle's pass on the same inputs; afterwards searches over the new
  partitioning follow the oracle's adaptive scan exactly.
"""

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import aps as oaps
from oracle import ivf as oivf
from oracle import maintenance as om

pytestmark = pytest.mark.gpu

LAMBDA_SIZE = [1, 50, 100, 150, 270, 300, 1000]
LAMBDA_COST = [10.0, 40.0, 60.0, 80.0, 380.0, 400.0, 2000.0]


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _pairs_index(metric, seed):
    """Partitions made of two nearby groups each, far from every other pair,
    plus tiny stray partitions next to some pairs.  Returns (X, assign, hits)."""
    rng = np.random.default_rng(seed)
    d = 32
    plan = [("hot", 150, 150)] * 8 + [("hot", 270, 30)] * 2 + [("cold", 50, 50)] * 10
    rows, assign, hits = [], [], []
    centres = rng.standard_normal((len(plan), d)) * 4.0
    if metric == "ip":
        centres = _unit(centres)
    sep, noise, stray_off = (1.0, 0.05, 3.0) if metric == "l2" else (0.08, 0.004, 0.25)
    for p, (kind, na, nb) in enumerate(plan):
        u = _unit(rng.standard_normal(d))
        a = centres[p] - 0.5 * sep * u
        b = centres[p] + 0.5 * sep * u
        blk = np.vstack([a + noise * rng.standard_normal((na, d)), b + noise * rng.standard_normal((nb, d))])
        rows.append(blk)
        assign += [p] * (na + nb)
        hits.append(900 if kind == "hot" else 50)
    # strays: four next to cold pairs, one next to a hot pair (10 rows, never visited)
    for host in (10, 12, 14, 16, 0):
        w = _unit(rng.standard_normal(d))
        c = centres[host] + stray_off * w
        rows.append(c + noise * rng.standard_normal((10, d)))
        assign += [len(hits)] * 10
        hits.append(0)
    X = np.vstack(rows).astype(np.float32)
    if metric == "ip":
        X = _unit(X).astype(np.float32)
    return X, np.asarray(assign, dtype=np.int32), np.asarray(hits, dtype=np.int64)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_maintenance_pass_matches_the_oracle(metric):
    X, assign, hits = _pairs_index(metric, seed=3 if metric == "l2" else 4)
    print(f"[build] pairs index {metric}: {X.shape[0]} rows, {hits.size} partitions", flush=True)
    idx = gu.build(X, metric=metric, nlist=int(hits.size), storage="bf16", assign=gu.to_dev(assign))
    try:
        before = gu.oracle_view(idx, X)
        assert (before.assign == assign).all()
        prm = om.MaintainParams(tau=0.2, alpha=1.0, refine_radius=1, refine_iters=1, split_iters=8,
                                min_split_size=2, merge_below=20)
        lam = om.Latency(LAMBDA_SIZE, LAMBDA_COST)
        part_o, C_o, dec_o = om.maintain(X, before.assign, before.C, hits, 1000, lam, prm, metric)
        rep, dec = idx.maintain(LAMBDA_SIZE, LAMBDA_COST, tau=prm.tau, alpha=prm.alpha,
                                refine_radius=prm.refine_radius, refine_iters=prm.refine_iters,
                                split_iters=prm.split_iters, min_split_size=prm.min_split_size,
                                merge_below=prm.merge_below, hits=hits, window=1000)
        print(f"[maintain] {rep}", flush=True)
        # the scenario exercises every branch of the workflow
        kinds = [(d.action, d.committed) for d in dec_o]
        assert kinds.count(("split", True)) == 8 and kinds.count(("split", False)) == 2
        assert kinds.count(("merge", True)) == 4
        assert [(d["partition"], ["split", "merge"][d["action"]], bool(d["committed"])) for d in dec] == \
            [(d.partition, d.action, d.committed) for d in dec_o]
        for a, b in zip(dec, dec_o):
            assert a["estimate"] == pytest.approx(b.estimate, rel=1e-9, abs=1e-9)
            assert a["verified"] == pytest.approx(b.verified, rel=1e-9, abs=1e-9)
        assert rep["splits"] == 8 and rep["deletes"] == 4
        assert rep["nlist_before"] == hits.size and rep["nlist_after"] == C_o.shape[0]
        after = gu.oracle_view(idx, X)
        assert after.nlist == C_o.shape[0]
        assert (after.assign == part_o).all(), np.nonzero(after.assign != part_o)[0][:10]
        np.testing.assert_allclose(after.C, C_o, atol=2e-5)
        hits_now, window = idx.access_stats()
        assert window == 0 and (hits_now == 0).all()
        # searches over the new partitioning follow the oracle
        rng = np.random.default_rng(5)
        Q = (X[rng.choice(X.shape[0], 200, replace=False)] +
             (0.05 if metric == "l2" else 0.004) * rng.standard_normal((200, X.shape[1]))).astype(np.float32)
        if metric == "ip":
            Q = _unit(Q).astype(np.float32)
        gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.25)
        order, h = idx.candidates(gu.to_dev(Q), 0.25)
        parity.check_aps(X, Q, after, gi, gv, ns, rec, order.cpu().numpy(), h.cpu().numpy(), metric, 0.25, 0.9, 10)
        bi, bv, _, _ = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.25, scan_mode="batched",
                                 scan_dtype="bf16", rerank_factor=4)
        id_to_row = {i: i for i in range(X.shape[0])}
        for i in range(0, 200, 10):
            tv = parity.true_values(Q[i], X, id_to_row, bi[i], metric)
            assert (np.abs(bv[i] - tv) <= parity.value_tol(Q[i], X, metric, tv)).all()
    finally:
        idx.free()


@pytest.fixture(scope="module")
def counted():
    spec = synth.MixtureSpec(key=61, n=20_000, d=32, n_components=40, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 300)
    idx = gu.build(X, metric="l2", nlist=64, storage="bf16", kmeans_iters=5, seed=2)
    ps = gu.oracle_view(idx, X)
    yield X, Q, idx, ps
    idx.free()


def test_counters_follow_fixed_nprobe(counted):
    X, Q, idx, ps = counted
    idx.access_stats(reset=True)
    gu.search(idx, Q, k=10, nprobe=6)
    hits, window = idx.access_stats(reset=True)
    assert window == Q.shape[0]
    want = np.zeros(ps.nlist, dtype=np.int64)
    ties = 0
    for i in range(Q.shape[0]):
        vals, order = oivf.centroid_ranking(Q[i], ps.C, "l2")
        want[order[:6]] += 1
        ks = np.sort(vals)
        if abs(ks[6] - ks[5]) <= 1e-5 * max(ks[5], 1e-30):
            ties += 1
    assert np.abs(hits - want).sum() <= 2 * ties, (hits, want)
    after, w2 = idx.access_stats()
    assert w2 == 0 and (after == 0).all()


def test_counters_follow_adaptive_scanning(counted):
    X, Q, idx, ps = counted
    idx.access_stats(reset=True)
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.1)
    hits, window = idx.access_stats(reset=True)
    assert window == Q.shape[0] and hits.sum() == ns.sum()
    order, h = idx.candidates(gu.to_dev(Q), 0.1)
    order, h = order.cpu().numpy(), h.cpu().numpy()
    table = oaps.CapTable(X.shape[1])
    params = oaps.APSParams(k=10, recall_target=0.9, f_M=0.1, metric="l2")
    want = np.zeros(ps.nlist, dtype=np.int64)
    dev = hits.copy()
    left_out = 0
    for i in range(Q.shape[0]):
        res = oaps.aps_search_one(ps, Q[i], params, table)
        m = int(ns[i])
        if res.m != m:
            assert parity.replay_margin(res, 0.9, 0.01, max(res.m, m)), f"query {i}: device {m}, oracle {res.m}"
        elif set(order[i, :m].tolist()) != set(res.order[:m].tolist()):
            # must be a near-tie in the candidate order (raises otherwise)
            assert not parity.check_candidate_order(Q[i], ps.C, 0.1, "l2", order[i], h[i])
        else:
            want[res.order[:m]] += 1
            continue
        dev[order[i, :m]] -= 1  # a query decided within the margin: left out on both sides
        left_out += 1
    assert left_out <= 0.02 * Q.shape[0]
    assert (dev == want).all(), np.nonzero(dev != want)[0]
    # the batched path counts the partitions it committed as well
    _, _, bns, _ = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.1, scan_mode="batched", scan_dtype="bf16",
                             rerank_factor=4)
    bh, bw = idx.access_stats(reset=True)
    assert bw == Q.shape[0] and bh.sum() == bns.sum()


def test_maintenance_with_the_index_counters(counted):
    """A pass driven by the index's own statistics: the estimates are the
    oracle's Eq. delta_split_est at A = hits / window read just before."""
    X, Q, idx0, ps = counted
    idx = gu.build(X, metric="l2", nlist=64, storage="f32", kmeans_iters=5, seed=2)
    try:
        idx.access_stats(reset=True)
        gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.1)
        hits, window = idx.access_stats()
        sizes = gu.oracle_view(idx, X).sizes()
        lam = om.Latency(LAMBDA_SIZE, [c * 0.01 for c in LAMBDA_COST])
        rep, dec = idx.maintain(LAMBDA_SIZE, [c * 0.01 for c in LAMBDA_COST], tau=0.0, alpha=0.9,
                                refine_radius=4, refine_iters=1, merge_below=0)
        dO = om.centroid_overhead_plus(64, lam)
        splits = [d for d in dec if d["action"] == 0]
        for d in splits:
            j = d["partition"]
            want = om.delta_split_estimate(dO, hits[j] / window, sizes[j], 0.9, lam)
            assert d["estimate"] == pytest.approx(want, rel=1e-9, abs=1e-12)
        tried = {d["partition"] for d in splits}
        for j in range(64):
            if j not in tried and sizes[j] >= 2:
                assert om.delta_split_estimate(dO, hits[j] / window, sizes[j], 0.9, lam) >= 0.0
        after = gu.oracle_view(idx, X)  # every vector present exactly once
        assert after.nlist == 64 + rep["splits"]
        gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.1)
        order, h = idx.candidates(gu.to_dev(Q), 0.1)
        parity.check_aps(X, Q, after, gi, gv, ns, rec, order.cpu().numpy(), h.cpu().numpy(), "l2", 0.1, 0.9, 10)
    finally:
        idx.free()


def test_two_level_maintenance_propagates_upward():
    """Maintenance of a two-level index acts on level 0 exactly as on the
    one-level index with the same level 0 (same decisions, partitions and
    centroids), keeps the level-1 centroids, and places every new level-0
    centroid in its nearest level-1 partition (Sec. 4.2: splits add, deletes
    remove a centroid at the parent level).  Searches then run on both
    levels and return the exact top-k over the partitions they scanned."""
    X, assign, hits = _pairs_index("l2", seed=3)
    print(f"[build] pairs index, one and two levels: {X.shape[0]} rows", flush=True)
    one = gu.build(X, metric="l2", nlist=int(hits.size), storage="bf16", assign=gu.to_dev(assign))
    C0, _, _ = one.export()
    two = gu.build(X, metric="l2", nlist=int(hits.size), n_levels=2, nlist_top=5, kmeans_iters=4, seed=3,
                   storage="bf16", centroids=C0, assign=gu.to_dev(assign))
    try:
        T_before, _ = two.export_level(1)
        kw = dict(tau=0.2, alpha=1.0, refine_radius=1, refine_iters=1, split_iters=8, min_split_size=2,
                  merge_below=20, hits=hits, window=1000)
        r1, d1 = one.maintain(LAMBDA_SIZE, LAMBDA_COST, **kw)
        r2, d2 = two.maintain(LAMBDA_SIZE, LAMBDA_COST, **kw)
        assert r1 == r2 and d1 == d2 and r2["splits"] == 8 and r2["deletes"] == 4
        a1, a2 = gu.oracle_view(one, X), gu.oracle_view(two, X)
        assert (a1.assign == a2.assign).all() and (a1.C == a2.C).all()
        T_after, top_of = two.export_level(1)
        assert (T_after.cpu().numpy() == T_before.cpu().numpy()).all()
        assert two.level_sizes() == [a2.nlist, 5, 0]
        bad = oivf.assignment_violations(a2.C, top_of.cpu().numpy().astype(np.int64), T_after.cpu().numpy(), "l2",
                                         rtol=1e-5)
        assert bad.size == 0
        rng = np.random.default_rng(5)
        Q = (X[rng.choice(X.shape[0], 200, replace=False)] + 0.05 * rng.standard_normal((200, X.shape[1]))
             ).astype(np.float32)
        gi, gv, ns, _ = gu.search(two, Q, k=10, recall_target=0.9, f_M=0.25, upper_recall_target=0.99,
                                  upper_f_M=0.5)
        order, h = two.candidates(gu.to_dev(Q), 0.25, upper_recall_target=0.99, upper_f_M=0.5)
        order = order.cpu().numpy()
        id_to_row = {i: i for i in range(X.shape[0])}
        for i in range(Q.shape[0]):
            dev = order[i][order[i] >= 0].astype(np.int64)
            ri, rv = oivf.scan_partitions(a2, Q[i], dev[: int(ns[i])], 10, "l2")
            parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")
    finally:
        one.free()
        two.free()


def test_latency_profile_on_this_gpu(counted):
    """lambda(s) measured on the device (the cost of one more partition of s
    of the index's vectors per query: eight-partition indexes searched with
    nprobe 8 and 1) is not negative and grows with s, for both scan paths,
    and the index it was taken from is left as it was."""
    X, Q, idx, ps = counted
    before = idx.stats()
    sizes = [64, 512, 2048]
    plain = idx.profile_latency(sizes, nq=1024, reps=2, k=10)
    batched = idx.profile_latency(sizes, nq=1024, reps=2, k=10, scan_mode="batched", scan_dtype="bf16",
                                  rerank_factor=4)
    print(f"[lambda] plain {plain} us, batched {batched} us per query", flush=True)
    assert (plain >= 0).all() and (batched >= 0).all()
    assert plain[-1] > plain[0] and batched[-1] > batched[0]
    assert idx.stats() == before
