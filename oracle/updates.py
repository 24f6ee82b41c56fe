"""Batched inserts and deletes, replayed on the CPU (Sec. 2.1 and Sec. 3).

Test infrastructure only (see the package docstring).

An insert walks the levels top-down to the nearest leaf partition and
appends the vector there; a delete finds the vector through the id map and
removes it (Sec. 3).  Centroids stay fixed: moving them is the maintenance
procedure's job (Sec. 4), not the update path's.

Batch rules (the paper leaves them open): a delete batch naming an id that
is not present, or naming an id twice, is rejected whole; an insert batch
whose ids repeat, or collide with a present id, is rejected whole.  Nearest
centroid ties go to the lower partition id.
"""

from __future__ import annotations

from typing import Optional

import numpy as np

from .ivf import PartitionedSet
from .knn import distances, sort_key

OK = 0
NOTFOUND = -3
DUPLICATE = -4


def nearest_partition(X: np.ndarray, C: np.ndarray, metric: str, allowed: Optional[np.ndarray] = None):
    """Index of the nearest centroid per row (FP64), lower id on ties."""
    D = distances(X, C, metric)
    key = sort_key(D, metric)
    if allowed is not None:
        key = np.where(allowed, key, np.inf)
    best = key.min(1, keepdims=True)
    # first column that attains the minimum = lowest id among exact ties
    return np.argmax(key == best, axis=1).astype(np.int64)


class ReplayIndex:
    def __init__(self, centroids: np.ndarray, metric: str, top_centroids: Optional[np.ndarray] = None,
                 top_assign: Optional[np.ndarray] = None):
        self.C = np.asarray(centroids, dtype=np.float32)
        self.metric = metric
        self.C1 = top_centroids
        self.top_assign = None if top_assign is None else np.asarray(top_assign, dtype=np.int64)
        self.vec = {}
        self.part = {}

    def load(self, X: np.ndarray, ids: np.ndarray, assign: np.ndarray):
        for i, x, a in zip(ids.tolist(), X, assign.tolist()):
            self.vec[i] = x
            self.part[i] = a

    def route(self, X: np.ndarray) -> np.ndarray:
        if self.C1 is None:
            return nearest_partition(X, self.C, self.metric)
        top = nearest_partition(X, self.C1, self.metric)
        out = np.empty(X.shape[0], dtype=np.int64)
        for t in np.unique(top):
            sel = np.nonzero(top == t)[0]
            allowed = (self.top_assign == t)[None, :]
            out[sel] = nearest_partition(X[sel], self.C, self.metric, allowed)
        return out

    def insert(self, X: np.ndarray, ids: np.ndarray) -> int:
        ids = [int(v) for v in ids]
        if len(set(ids)) != len(ids) or any(i in self.vec for i in ids):
            return DUPLICATE
        if not ids:
            return OK
        parts = self.route(X)
        for i, x, p in zip(ids, X, parts.tolist()):
            self.vec[i] = np.array(x, dtype=np.float32)
            self.part[i] = p
        return OK

    def delete(self, ids: np.ndarray) -> int:
        ids = [int(v) for v in ids]
        if len(set(ids)) != len(ids) or any(i not in self.vec for i in ids):
            return NOTFOUND
        for i in ids:
            del self.vec[i]
            del self.part[i]
        return OK

    def partitioned(self) -> PartitionedSet:
        ids = np.array(sorted(self.vec), dtype=np.int64)
        d = self.C.shape[1]
        X = np.stack([self.vec[i] for i in ids]) if ids.size else np.zeros((0, d), np.float32)
        assign = np.array([self.part[i] for i in ids], dtype=np.int64)
        return PartitionedSet(X, ids, assign, self.C)
