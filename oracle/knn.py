"""Exact k-nearest-neighbour search and recall@k (Sec. 2.1, problem statement).

Test infrastructure only (see the package docstring).

Conventions (the paper fixes neither):
* L2 results are *squared* Euclidean distances, ascending.
* Inner-product results are scores, descending.
* Ties are broken by the lower id.  Missing results (fewer than k candidates)
  are id -1 with distance +inf (L2) or -inf (IP).
"""

from __future__ import annotations

import numpy as np

# Above this many multiply-adds the squared distance is evaluated through the
# FP64 expansion |q|^2 - 2 q.x + |x|^2 instead of the literal sum of squared
# differences.  In FP64 the expansion's absolute error is at most
# ~d * 2^-53 * (|q|^2 + 2|q||x| + |x|^2), below 1e-10 relative for every
# workload here, far under the 1e-5 comparison tolerance; the pin tests check
# the two forms against each other on small inputs.
_DIRECT_LIMIT = 2e8


def l2_direct(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Sum over dimensions of (q_i - x_i)^2 in FP64, the definition written out."""
    Q64 = np.asarray(Q, dtype=np.float64)
    X64 = np.asarray(X, dtype=np.float64)
    out = np.empty((Q64.shape[0], X64.shape[0]))
    for i in range(Q64.shape[0]):
        diff = X64 - Q64[i]
        out[i] = np.einsum("ij,ij->i", diff, diff)
    return out


def l2_expanded(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    Q64 = np.asarray(Q, dtype=np.float64)
    X64 = np.asarray(X, dtype=np.float64)
    qq = np.einsum("ij,ij->i", Q64, Q64)
    xx = np.einsum("ij,ij->i", X64, X64)
    d = qq[:, None] + xx[None, :] - 2.0 * (Q64 @ X64.T)
    return np.maximum(d, 0.0)


def inner_product(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    return np.asarray(Q, dtype=np.float64) @ np.asarray(X, dtype=np.float64).T


def distances(Q: np.ndarray, X: np.ndarray, metric: str) -> np.ndarray:
    """[nq, n] FP64 squared L2 distances or inner products."""
    if metric == "ip":
        return inner_product(Q, X)
    if metric != "l2":
        raise ValueError(metric)
    work = float(Q.shape[0]) * X.shape[0] * X.shape[1]
    return l2_direct(Q, X) if work <= _DIRECT_LIMIT else l2_expanded(Q, X)


def sort_key(vals: np.ndarray, metric: str) -> np.ndarray:
    """Ascending key: distance for L2, negated score for IP."""
    return -vals if metric == "ip" else vals


def empty_value(metric: str) -> float:
    return -np.inf if metric == "ip" else np.inf


def select_topk(vals: np.ndarray, ids: np.ndarray, k: int, metric: str):
    """Best k of one row by (key, id) ascending: (ids int64 [k], vals f64 [k])."""
    out_i = np.full(k, -1, dtype=np.int64)
    out_v = np.full(k, empty_value(metric))
    n = vals.shape[0]
    if n == 0:
        return out_i, out_v
    key = sort_key(vals, metric)
    kk = min(k, n)
    if n > kk:
        thr = np.partition(key, kk - 1)[kk - 1]
        cand = np.nonzero(key <= thr)[0]
    else:
        cand = np.arange(n)
    order = np.lexsort((ids[cand], key[cand]))[:kk]
    out_i[:kk] = ids[cand[order]]
    out_v[:kk] = vals[cand[order]]
    return out_i, out_v


def merge_topk(a_ids, a_vals, b_ids, b_vals, k: int, metric: str):
    ids = np.concatenate([a_ids, b_ids])
    vals = np.concatenate([a_vals, b_vals])
    live = ids >= 0
    return select_topk(vals[live], ids[live], k, metric)


def knn_exact(X: np.ndarray, ids: np.ndarray, Q: np.ndarray, k: int, metric: str,
              row_block: int = 131072, query_block: int = 256):
    """Exact k-NN of every query over every row of X.

    Returns (ids int64 [nq, k], values f64 [nq, k]).
    """
    nq = Q.shape[0]
    ids = np.asarray(ids, dtype=np.int64)
    res_i = np.full((nq, k), -1, dtype=np.int64)
    res_v = np.full((nq, k), empty_value(metric))
    for q0 in range(0, nq, query_block):
        qb = Q[q0:q0 + query_block]
        cur_i = res_i[q0:q0 + qb.shape[0]]
        cur_v = res_v[q0:q0 + qb.shape[0]]
        for r0 in range(0, X.shape[0], row_block):
            D = distances(qb, X[r0:r0 + row_block], metric)
            rid = ids[r0:r0 + row_block]
            for j in range(qb.shape[0]):
                ti, tv = select_topk(D[j], rid, k, metric)
                cur_i[j], cur_v[j] = merge_topk(cur_i[j], cur_v[j], ti, tv, k, metric)
    return res_i, res_v


def recall_at_k(found: np.ndarray, truth: np.ndarray, k: int) -> np.ndarray:
    """|G n R| / k per query (Sec. 2.1); -1 entries never count."""
    out = np.empty(found.shape[0])
    for i in range(found.shape[0]):
        g = set(int(v) for v in truth[i, :k] if v >= 0)
        r = set(int(v) for v in found[i, :k] if v >= 0)
        out[i] = len(g & r) / float(k)
    return out
