"""Fixed-nprobe partition scan and the nearest-centroid assignment (Sec. 3).

Test infrastructure only (see the package docstring).

The index keeps disjoint partitions, each with a centroid (Sec. 3, "index
structure"); a query ranks the centroids and scans the vectors of the
nearest ones (Sec. 1 / Sec. 2.3).  The oracle takes the device index's
centroids and assignment as inputs so that it scans the same partitions.
"""

from __future__ import annotations

import numpy as np

from .knn import distances, select_topk, sort_key


class PartitionedSet:
    """Vectors grouped by partition: members[p] = row indices of partition p."""

    def __init__(self, X: np.ndarray, ids: np.ndarray, assign: np.ndarray, centroids: np.ndarray):
        self.X = X
        self.ids = np.asarray(ids, dtype=np.int64)
        self.assign = np.asarray(assign, dtype=np.int64)
        self.C = np.asarray(centroids)
        N = self.C.shape[0]
        order = np.argsort(self.assign, kind="stable")
        bounds = np.searchsorted(self.assign[order], np.arange(N + 1))
        self.members = [order[bounds[p]:bounds[p + 1]] for p in range(N)]

    @property
    def nlist(self) -> int:
        return self.C.shape[0]

    def sizes(self) -> np.ndarray:
        return np.array([m.shape[0] for m in self.members], dtype=np.int64)


def centroid_ranking(q: np.ndarray, C: np.ndarray, metric: str):
    """Centroid values (squared L2 or IP, FP64) and the order (key, id) ascending."""
    vals = distances(q[None, :], C, metric)[0]
    key = sort_key(vals, metric)
    order = np.lexsort((np.arange(C.shape[0]), key))
    return vals, order


def scan_partitions(ps: PartitionedSet, q: np.ndarray, parts, k: int, metric: str):
    """Exact top-k over the union of the given partitions' vectors."""
    parts = list(parts)
    if parts:
        rows = np.concatenate([ps.members[p] for p in parts])
    else:
        rows = np.zeros(0, dtype=np.int64)
    if rows.shape[0] == 0:
        return select_topk(np.zeros(0), np.zeros(0, dtype=np.int64), k, metric)
    vals = distances(q[None, :], ps.X[rows], metric)[0]
    return select_topk(vals, ps.ids[rows], k, metric)


def ivf_search(ps: PartitionedSet, Q: np.ndarray, k: int, nprobe: int, metric: str):
    """Scan the nprobe nearest partitions of every query.

    Returns (ids [nq, k], values [nq, k], probed partitions [nq, nprobe]).
    """
    nq = Q.shape[0]
    nprobe = min(nprobe, ps.nlist)
    out_i = np.empty((nq, k), dtype=np.int64)
    out_v = np.empty((nq, k))
    probes = np.empty((nq, nprobe), dtype=np.int64)
    for i in range(nq):
        _, order = centroid_ranking(Q[i], ps.C, metric)
        probes[i] = order[:nprobe]
        out_i[i], out_v[i] = scan_partitions(ps, Q[i], probes[i], k, metric)
    return out_i, out_v, probes


def assignment_violations(X: np.ndarray, assign: np.ndarray, C: np.ndarray, metric: str,
                          rtol: float = 1e-6, block: int = 65536) -> np.ndarray:
    """Rows whose partition is not the nearest centroid, beyond a near-tie.

    L2: the assigned centroid's squared distance may exceed the minimum by at
    most rtol relative.  IP: the assigned score may fall short of the maximum
    by at most rtol * (|x| * max|c|).
    """
    bad = []
    cn = np.sqrt((np.asarray(C, dtype=np.float64) ** 2).sum(1)).max()
    for r0 in range(0, X.shape[0], block):
        D = distances(X[r0:r0 + block], C, metric)
        a = np.asarray(assign[r0:r0 + block], dtype=np.int64)
        mine = D[np.arange(D.shape[0]), a]
        if metric == "ip":
            best = D.max(1)
            xn = np.sqrt((np.asarray(X[r0:r0 + block], dtype=np.float64) ** 2).sum(1))
            viol = best - mine > rtol * xn * cn
        else:
            best = D.min(1)
            viol = mine - best > rtol * np.maximum(best, 1e-30)
        bad.append(np.nonzero(viol)[0] + r0)
    return np.concatenate(bad) if bad else np.zeros(0, dtype=np.int64)
