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
