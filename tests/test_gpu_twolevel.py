"""Two-level index on the device against the oracle's two-level search.

Level 1 holds the level-0 centroids in its own partitions; a search runs
adaptive scanning over level 1 to pick the level-0 candidates, then over
level 0.  With the upper level set to scan everything exactly (target 1,
fraction 1) the result must equal single-level scanning; with the paper's
settings (0.99, 25%) the device must follow the oracle's procedure query by
query, up to decisions within the floating-point margin.
"""

import math

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import aps as oaps
from oracle import ivf as oivf
from oracle import knn as oknn
from oracle import twolevel as otl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def two_level():
    spec = synth.MixtureSpec(key=41, n=60_000, d=32, n_components=60, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 200)
    print("[build] two-level 60k x 32, 400 leaves under 8 top partitions", flush=True)
    idx = gu.build(X, metric="l2", nlist=400, n_levels=2, nlist_top=8, kmeans_iters=5, seed=7)
    leaves = gu.oracle_view(idx, X)
    from paper_2506_03437_amd import quake_export_top
    C1, top_of = quake_export_top(idx.handle, X.shape[1], 8)
    tl = otl.TwoLevelSet(leaves, top_of.cpu().numpy().astype(np.int64), C1.cpu().numpy())
    yield X, Q, idx, tl
    idx.free()


def test_top_partitioning_is_nearest(two_level):
    X, Q, idx, tl = two_level
    bad = oivf.assignment_violations(tl.leaves.C, tl.top.assign, tl.top.C, "l2", rtol=1e-5)
    assert bad.size == 0


def test_exact_upper_level_equals_single_level(two_level):
    X, Q, idx, tl = two_level
    gi, gv, ns, _ = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, upper_recall_target=1.0, upper_f_M=1.0)
    table = oaps.CapTable(X.shape[1])
    params = oaps.APSParams(k=10, recall_target=0.9, f_M=0.05, metric="l2")
    id_to_row = {i: i for i in range(X.shape[0])}
    for i in range(Q.shape[0]):
        res = oaps.aps_search_one(tl.leaves, Q[i], params, table)
        ri, rv = oivf.scan_partitions(tl.leaves, Q[i], res.order[: ns[i]], 10, "l2")
        parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")


def test_paper_settings_follow_the_oracle(two_level):
    """Query by query, over the device's own candidate list (exported by
    quake_candidates from the device's level-1 search): the results are
    exactly the top-k over the partitions the device scanned; the list is
    the oracle's level-1 result up to near-ties or level-1 decisions within
    the margin; c_0, the order and h are the oracle's over that list; and
    the stop count and recall estimate replay the oracle's level-0 APS over
    the device's order except decisions within the margin."""
    X, Q, idx, tl = two_level
    kw = dict(upper_recall_target=0.99, upper_f_M=0.25)
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, **kw)
    order, h = idx.candidates(gu.to_dev(Q), 0.05, **kw)
    order, h = order.cpu().numpy(), h.cpu().numpy()
    table = oaps.CapTable(X.shape[1])
    M0 = oaps.candidate_count(0.05, tl.leaves.nlist)
    assert order.shape[1] == M0
    upper = oaps.APSParams(k=M0, recall_target=0.99, f_M=0.25, metric="l2")
    lower = oaps.APSParams(k=10, recall_target=0.9, f_M=0.05, metric="l2")
    id_to_row = {i: i for i in range(X.shape[0])}
    set_margin = stop_margin = 0
    for i in range(Q.shape[0]):
        dev = order[i][order[i] >= 0].astype(np.int64)
        hdev = h[i][: dev.size]
        m = int(ns[i])
        assert 1 <= m <= dev.size
        ri, rv = oivf.scan_partitions(tl.leaves, Q[i], dev[:m], 10, "l2")
        parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")
        r1 = oaps.aps_search_one(tl.top, Q[i], upper, table)
        if set(dev.tolist()) != set(r1.ids[r1.ids >= 0].tolist()):
            assert parity.level1_set_explained(Q[i], tl.leaves.C, dev.tolist(), r1, 0.99), f"query {i}: level-1 set"
            set_margin += 1
        if not parity.check_candidate_order(Q[i], tl.leaves.C, 0.05, "l2", dev, hdev, cands=dev):
            set_margin += 1
            continue
        vals = oknn.distances(Q[i][None], tl.leaves.C, "l2")[0]
        h_ref = oaps.bisector_distances(Q[i], tl.leaves.C, vals, int(dev[0]), dev[1:], "l2")
        r0 = oaps.aps_search_one(tl.leaves, Q[i], lower, table, order=dev, h=h_ref)
        if r0.m != m:
            assert parity.replay_margin(r0, 0.9, 0.01, max(r0.m, m)), f"query {i}: device {m}, oracle {r0.m}"
            stop_margin += 1
        else:
            assert abs(rec[i] - r0.steps[-1].recall) < 1e-4, f"query {i}: recall estimate"
    assert set_margin + stop_margin <= 0.03 * Q.shape[0], (set_margin, stop_margin)
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q, 10, "l2")
    assert oknn.recall_at_k(gi, truth, 10).mean() >= 0.85


def test_two_level_nprobe_with_exact_upper_level(two_level):
    X, Q, idx, tl = two_level
    gi, gv, ns, _ = gu.search(idx, Q, k=10, nprobe=12, upper_recall_target=1.0, upper_f_M=1.0)
    assert (ns == 12).all()
    ri, rv, _ = oivf.ivf_search(tl.leaves, Q, 10, 12, "l2")
    parity.check_all(Q, X, tl.leaves.ids, gi, gv, ri, rv, "l2", 10)


def test_two_level_insert_routes_top_down(two_level):
    X, Q, idx, tl = two_level
    rng = np.random.default_rng(3)
    B = (X[rng.choice(X.shape[0], 300)] + 0.05 * rng.standard_normal((300, X.shape[1]))).astype(np.float32)
    bid = np.arange(1_000_000, 1_000_300, dtype=np.int64)
    idx.insert(gu.to_dev(B), gu.to_dev(bid))
    from oracle import updates as oupd
    r = oupd.ReplayIndex(tl.leaves.C, "l2", top_centroids=tl.top.C, top_assign=tl.top.assign)
    expect = r.route(B)
    C, eids, epart = idx.export()
    got = dict(zip(eids.cpu().numpy().tolist(), epart.cpu().numpy().tolist()))
    mism = [i for i, e in zip(bid.tolist(), expect.tolist()) if got[i] != e]
    assert len(mism) <= 1, mism
    idx.delete(gu.to_dev(bid))
