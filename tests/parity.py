"""Comparison rules between the device search and the CPU oracle.

Tolerances (derived from the FP32 arithmetic of the device path):
* Distances: the device sums squared differences (or products) in FP32 with
  blocked partial sums; the relative error of a squared L2 distance is at
  most about (d/8 + 4) * 2^-24 < 1e-5 for d <= 768, so reported L2
  distances must agree with the FP64 value within 1e-5 relative.  For inner
  products the bound is relative to |q| |x| (the sum of |q_i x_i|), so the
  tolerance is 1e-5 * |q| * max |x|.
* Ids: every oracle neighbour whose key is clearly inside the k-th key
  (by more than the tolerance) must be returned, and no returned id may be
  clearly outside it; ids within the tolerance of the k-th key are ties
  that either side may order differently.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import knn

RTOL = 1e-5


def key_of(vals, metric):
    return -np.asarray(vals) if metric == "ip" else np.asarray(vals)


def value_tol(q, X, metric, vals):
    if metric == "ip":
        scale = float(np.linalg.norm(q.astype(np.float64))) * float(np.sqrt((X.astype(np.float64) ** 2).sum(1)).max())
        return np.full(np.shape(vals), RTOL * scale)
    return RTOL * np.maximum(np.abs(np.asarray(vals, dtype=np.float64)), 1e-30)


def true_values(q, X, id_to_row, ids, metric):
    rows = np.array([id_to_row[int(i)] for i in ids], dtype=np.int64)
    if rows.size == 0:
        return np.zeros(0)
    return knn.distances(q[None, :], X[rows], metric)[0]


def check_topk(q, X, id_to_row, gpu_ids, gpu_vals, ref_ids, ref_vals, metric, k, where=""):
    """Raise AssertionError with a message when the device result breaks the rules."""
    gpu_ids = np.asarray(gpu_ids)
    gpu_vals = np.asarray(gpu_vals, dtype=np.float64)
    n_ref = int((ref_ids >= 0).sum())
    n_gpu = int((gpu_ids >= 0).sum())
    assert n_gpu == n_ref, f"{where}: {n_gpu} results, oracle has {n_ref}"
    assert (gpu_ids[n_gpu:] == -1).all(), f"{where}: ids after the last result must be -1"
    if n_ref == 0:
        return
    live = gpu_ids[:n_gpu]
    assert len(set(live.tolist())) == n_gpu, f"{where}: repeated ids {live}"
    tv = true_values(q, X, id_to_row, live, metric)
    tol = value_tol(q, X, metric, tv)
    err = np.abs(gpu_vals[:n_gpu] - tv)
    assert (err <= tol).all(), f"{where}: distance error {err.max():.3e} > tol {tol[np.argmax(err - tol)]:.3e}"
    gk = key_of(gpu_vals[:n_gpu], metric)
    assert (np.diff(gk) >= 0).all(), f"{where}: results are not sorted"
    rk = key_of(ref_vals[:n_ref], metric)
    kth = rk[-1]
    ktol = float(value_tol(q, X, metric, np.array([ref_vals[n_ref - 1]]))[0])
    core = set(int(i) for i, kk in zip(ref_ids[:n_ref], rk) if kk < kth - ktol)
    missing = core - set(live.tolist())
    assert not missing, f"{where}: missing clear neighbours {sorted(missing)[:5]}"
    tk = key_of(tv, metric)
    outside = [int(i) for i, kk in zip(live, tk) if kk > kth + ktol]
    assert not outside, f"{where}: returned ids clearly beyond the k-th: {outside[:5]}"


def check_all(Q, X, ids, gpu_ids, gpu_vals, ref_ids, ref_vals, metric, k):
    id_to_row = {int(i): r for r, i in enumerate(np.asarray(ids).tolist())}
    bad = []
    for i in range(Q.shape[0]):
        try:
            check_topk(Q[i], X, id_to_row, gpu_ids[i], gpu_vals[i], ref_ids[i], ref_vals[i], metric, k, f"query {i}")
        except AssertionError as e:
            bad.append(str(e))
    assert not bad, f"{len(bad)} of {Q.shape[0]} queries differ; first: {bad[:3]}"


def check_candidate_order(q, C, f_M, metric, order, h_gpu, cands=None):
    """The device order is a valid APS order for the oracle, up to near-ties.

    With ``cands`` (the candidate set a level above handed over) the set is
    taken as given and only c_0, the order and h are checked."""
    from oracle import aps as oaps
    o_ref, h_ref = oaps.aps_order(q, C, f_M, metric, cands=cands)
    vals = knn.distances(q[None], C, metric)[0]
    key = knn.sort_key(vals, metric)
    scale = abs(key[o_ref[0]]) if metric == "l2" else float(np.linalg.norm(q)) * float(np.linalg.norm(C, axis=1).max())
    tol = 1e-5 * max(scale, 1e-30) + 1e-6
    # same candidate set except near-ties at the M-th place
    if cands is not None:
        assert set(order.tolist()) == set(o_ref.tolist()), "candidate set differs from the one handed over"
    elif set(order.tolist()) != set(o_ref.tolist()):
        ks = np.sort(key)
        M = o_ref.shape[0]
        assert M < key.shape[0] and abs(ks[M] - ks[M - 1]) <= tol, "candidate set differs"
        return False
    if order[0] != o_ref[0]:
        assert abs(key[order[0]] - key[o_ref[0]]) <= tol, "c0 differs"
        return False
    h_of = oaps.bisector_distances(q, C, vals, int(order[0]), order[1:].astype(np.int64), metric)
    # non-decreasing in the oracle's h, up to FP32 rounding of h
    htol = 1e-4 * max(float(np.abs(h_of).max(initial=0.0)), 1e-6)
    assert (np.diff(h_of) >= -htol).all(), "device order is not ascending in h"
    np.testing.assert_allclose(h_gpu[1:], h_of, atol=htol)
    return True


def replay_margin(res, tau_r, tau_rho, upto):
    """True when a stop or recompute decision up to step `upto` is too close to call."""
    for st in res.steps[:upto]:
        if abs(st.recall - tau_r) < 1e-4:
            return True
        if math.isfinite(st.recompute_gap) and abs(st.recompute_gap) < 1e-5 * max(st.rho, 1e-30):
            return True
    return False


def scan_filtered(ps, q, parts, k, metric, attr, mask):
    """Exact top-k over the rows of the given partitions whose label bits
    share a bit with `mask`."""
    from oracle import ivf as oivf
    rows = np.concatenate([ps.members[int(p)] for p in parts]) if len(parts) else np.zeros(0, dtype=np.int64)
    rows = rows[(np.asarray(attr, dtype=np.uint64)[rows] & np.uint64(int(mask))) != 0]
    sub = oivf.PartitionedSet(ps.X[rows], ps.ids[rows], np.zeros(rows.shape[0], dtype=np.int64), ps.C[:1])
    return oivf.scan_partitions(sub, q, [0], k, metric)


def check_aps(X, Q, ps, gi, gv, ns, rec, order, h, metric, f_M, tau_r, k=10, rows=None, estimator="aps",
              attr=None, masks=None):
    """Adaptive-scan parity for the queries `rows` (default all) of a device
    search: the results are the top-k over the partitions the device
    scanned, the candidate order is a valid APS order, and the stop count
    and recall estimate replay the oracle's, except decisions within the
    margins (at most 1% of the queries).  `estimator` names the variant the
    device ran: "aps" (threshold recompute, table), "aps-r" (every
    partition, table) or "aps-rp" (every partition, direct evaluation).
    With `attr` (label bits of every row of ps) and `masks` (one per query)
    the search was filtered."""
    from oracle import aps as oaps
    from oracle import ivf as oivf
    rows = np.arange(Q.shape[0]) if rows is None else np.asarray(rows)
    table = oaps.ExactCap(X.shape[1]) if estimator == "aps-rp" else oaps.CapTable(X.shape[1])
    params = oaps.APSParams(k=k, recall_target=tau_r, f_M=f_M, metric=metric,
                            recompute_every=estimator in ("aps-r", "aps-rp"))
    id_to_row = {int(i): r for r, i in enumerate(ps.ids.tolist())}
    margin = 0
    ordered = 0
    for j, i in enumerate(rows.tolist()):
        m = int(ns[i])
        assert 1 <= m <= order.shape[1]
        # results: exactly the top-k over the partitions the device scanned
        if attr is None:
            ri, rv = oivf.scan_partitions(ps, Q[i], order[j, :m], k, metric)
        else:
            ri, rv = scan_filtered(ps, Q[i], order[j, :m], k, metric, attr, masks[i])
        check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, metric, k, f"query {i}")
        if not check_candidate_order(Q[i], ps.C, f_M, metric, order[j], h[j]):
            continue
        ordered += 1
        vals = knn.distances(Q[i][None], ps.C, metric)[0]
        h_ref = oaps.bisector_distances(Q[i], ps.C, vals, int(order[j, 0]), order[j, 1:].astype(np.int64), metric)
        res = oaps.aps_search_one(ps, Q[i], params, table, order=order[j].astype(np.int64), h=h_ref, attr=attr,
                                  mask=None if masks is None else int(masks[i]))
        if res.m != m:
            assert replay_margin(res, tau_r, 0.01, max(res.m, m)), f"query {i}: device scanned {m}, oracle {res.m}"
            margin += 1
        else:
            assert abs(rec[i] - res.steps[-1].recall) < 1e-4, f"query {i}: recall estimate {rec[i]} vs {res.steps[-1].recall}"
    # every query left out was shown to be a near-tie (candidate set or c_0)
    # or a decision within the margin; these bound how many may be
    assert ordered >= 0.95 * rows.size, f"{rows.size - ordered} of {rows.size} queries with a near-tie candidate set"
    assert margin <= max(2, 0.01 * rows.size), f"{margin} queries decided within the margin"


def level1_set_explained(q, C0, dev_set, r1, tau1, metric="l2"):
    """A device level-0 candidate set that differs from the oracle's level-1
    result must differ only in centroids tied (within 1e-5) with the M0-th
    one, or the oracle's level-1 search must have decided within the margin."""
    ref = r1.ids[r1.ids >= 0]
    D = knn.distances(q[None], C0, metric)[0]
    key = -D if metric == "ip" else D
    kth = float(key[ref].max())
    diff = set(dev_set) ^ set(ref.tolist())
    if all(abs(float(key[j]) - kth) <= 1e-5 * max(abs(kth), 1e-30) for j in diff):
        return True
    return replay_margin(r1, tau1, 0.01, r1.m)
