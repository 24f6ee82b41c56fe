"""The 50M x 128 two-level FP16 workload's code path at reduced size.

Same shape parameters as the full workload except the row count (2M
instead of 50M, so a leaf holds 40 rows on average instead of 1,000):
50,000 generator-defined leaves whose centres are the level-0 centroids
(each row stored in its nearest), 64 top partitions, L2, an FP16 copy with
FP32 rerank, f_M = 0.015 so that the level-1 search returns M0 = 750
level-0 candidates (a level-1 result list past 256 entries), and one
65,536-query call per path.

* The device's level-0 candidate lists (quake_candidates with the level-1
  settings 0.99 / 25%) are the oracle's level-1 results up to near-ties or
  level-1 decisions within the margin, and c_0, the order and h over each
  list are the oracle's.
* Plain FP32 path: on a seeded sample, the results are exactly the top-k
  over the partitions scanned and the stop counts replay the oracle's
  level-0 adaptive scan over the device's list.
* Batched FP16 path: the reranked distances are the exact FP32 distances of
  the returned ids, and recall@10 against FP64 ground truth stays within
  0.005 of the FP32 path at targets 0.8, 0.9 and 0.95.
"""

from dataclasses import replace

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

N_ROWS = 2_000_000
F_M = 0.015
UPPER = dict(upper_recall_target=0.99, upper_f_M=0.25)


@pytest.fixture(scope="module")
def two_level_f16():
    base = synth.get_workload("two-level-50m-d128-f16")
    ls = replace(base.leaves, mixture=replace(base.leaves.mixture, n=N_ROWS))
    centres, _, X = synth.leaf_spec_database(ls, threads=8)
    Q = synth.leaf_spec_queries(ls, X, base.nq, base.query_noise)
    print(f"[build] reduced {base.name}: n={N_ROWS} leaves={base.nlist} top={base.nlist_top} "
          f"queries={base.nq}", flush=True)
    idx = gu.build(X, metric="l2", nlist=base.nlist, storage="f16", n_levels=2, nlist_top=base.nlist_top,
                   centroids=gu.to_dev(centres), kmeans_iters=10, seed=1)
    leaves = gu.oracle_view(idx, X)
    from paper_2506_03437_amd import quake_export_top
    C1, top_of = quake_export_top(idx.handle, X.shape[1], base.nlist_top)
    tl = otl.TwoLevelSet(leaves, top_of.cpu().numpy().astype(np.int64), C1.cpu().numpy())
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(base.nq, 160, replace=False))
    yield X, Q, idx, tl, sample
    idx.free()


def test_rows_sit_in_their_nearest_leaf(two_level_f16):
    X, Q, idx, tl, sample = two_level_f16
    rng = np.random.default_rng(2)
    rows = rng.choice(X.shape[0], 20_000, replace=False)
    bad = oivf.assignment_violations(X[rows], tl.leaves.assign[rows], tl.leaves.C, "l2")
    assert bad.size == 0, rows[bad[:5]]


def test_level0_candidates_follow_the_oracle(two_level_f16):
    X, Q, idx, tl, sample = two_level_f16
    order, h = idx.candidates(gu.to_dev(Q[sample]), F_M, **UPPER)
    order, h = order.cpu().numpy(), h.cpu().numpy()
    M0 = oaps.candidate_count(F_M, tl.leaves.nlist)
    assert M0 == 750 and order.shape[1] == M0
    table = oaps.CapTable(X.shape[1])
    upper = oaps.APSParams(k=M0, recall_target=0.99, f_M=0.25, metric="l2")
    margin = 0
    for j, i in enumerate(sample[:48].tolist()):
        dev = order[j][order[j] >= 0].astype(np.int64)
        r1 = oaps.aps_search_one(tl.top, Q[i], upper, table)
        if set(dev.tolist()) != set(r1.ids[r1.ids >= 0].tolist()):
            assert parity.level1_set_explained(Q[i], tl.leaves.C, dev.tolist(), r1, 0.99), f"query {i}"
            margin += 1
        if not parity.check_candidate_order(Q[i], tl.leaves.C, F_M, "l2", dev, h[j][: dev.size], cands=dev):
            margin += 1  # c_0 within the tie tolerance of the oracle's
    assert margin <= 2, margin


def test_plain_fp32_follows_the_oracle(two_level_f16):
    X, Q, idx, tl, sample = two_level_f16
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=F_M, **UPPER)
    order, h = idx.candidates(gu.to_dev(Q[sample]), F_M, **UPPER)
    order, h = order.cpu().numpy(), h.cpu().numpy()
    table = oaps.CapTable(X.shape[1])
    lower = oaps.APSParams(k=10, recall_target=0.9, f_M=F_M, metric="l2")
    id_to_row = {i: i for i in range(X.shape[0])}
    stop_margin = 0
    for j, i in enumerate(sample[:64].tolist()):
        dev = order[j][order[j] >= 0].astype(np.int64)
        m = int(ns[i])
        assert 1 <= m <= dev.size
        ri, rv = oivf.scan_partitions(tl.leaves, Q[i], dev[:m], 10, "l2")
        parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")
        vals = oknn.distances(Q[i][None], tl.leaves.C, "l2")[0]
        h_ref = oaps.bisector_distances(Q[i], tl.leaves.C, vals, int(dev[0]), dev[1:], "l2")
        r0 = oaps.aps_search_one(tl.leaves, Q[i], lower, table, order=dev, h=h_ref)
        if r0.m != m:
            assert parity.replay_margin(r0, 0.9, 0.01, max(r0.m, m)), f"query {i}: device {m}, oracle {r0.m}"
            stop_margin += 1
        else:
            assert abs(rec[i] - r0.steps[-1].recall) < 1e-4, f"query {i}: recall estimate"
    assert stop_margin <= 2, stop_margin


def test_batched_f16_path(two_level_f16):
    X, Q, idx, tl, sample = two_level_f16
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q[sample], 10, "l2")
    id_to_row = {i: i for i in range(X.shape[0])}
    for tau in (0.8, 0.9, 0.95):
        fi, _, fns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=F_M, **UPPER)
        bi, bv, bns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=F_M, scan_mode="batched",
                                   scan_dtype="f16", rerank_factor=6, **UPPER)
        rf = oknn.recall_at_k(fi[sample], truth, 10).mean()
        rb = oknn.recall_at_k(bi[sample], truth, 10).mean()
        print(f"[recall] tau {tau}: fp32 {rf:.4f} f16+rerank {rb:.4f} "
              f"(partitions {fns.mean():.2f} / {bns.mean():.2f})", flush=True)
        assert rb >= rf - 0.005, (tau, rf, rb)
        for i in sample[::8].tolist():
            live = bi[i][bi[i] >= 0]
            assert live.size == 10
            tv = parity.true_values(Q[i], X, id_to_row, live, "l2")
            assert (np.abs(bv[i] - tv) <= parity.value_tol(Q[i], X, "l2", tv)).all()
            assert (np.diff(bv[i]) >= 0).all()
