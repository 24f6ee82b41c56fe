"""Product quantization of the stored vectors and the compressed scan (Sec. 8,
"Vector Compression": the paper names product quantization as the way to
cut scan cost, with lambda re-profiled on the compressed scan, and leaves
the design open).

Test infrastructure only (see the package docstring).

Product quantization (Jegou, Douze and Schmid, IEEE TPAMI 33(1), 2011): the
d dimensions are split into M subspaces of d / M consecutive dimensions; in
each, a codebook of 256 codewords; a vector is stored as the M indices of
its nearest codewords.  A query is compared with a stored vector through
the vector its codes decode to ("asymmetric distance": the query is not
quantized).  In a partitioned index the codes quantize each row's residual
to its partition's centroid (the paper's IVFADC), so a row decodes to
centroid + decoded residual.

Readings of points the paper leaves open (each is also listed with its
reason in the design notes):
* P1  the codes quantize residuals to the partition centroid, with one
      codebook for the whole index; a row whose partition or centroid
      changes (split, merge, refinement) is encoded again.  (Codes of the
      vectors themselves spend the 256 codewords of a subspace on the
      spread of the cluster centres and cannot rank rows inside one
      cluster.)
* P2  each subspace's codebook is trained by Lloyd's k-means in squared
      Euclidean distance (for either metric) over residuals, started from
      256 distinct rows; a codeword left without rows keeps its value.  A
      row's code in a subspace is its nearest codeword, ties to the lower
      index.
* P3  the scan scores a row by the asymmetric value: squared L2 distance or
      inner product of the query and the row's decoded vector.
* P4  APS runs unchanged on the scanned scores: rho comes from the k-th
      best score so far; the scan keeps the best r * k rows by score, and
      once the search stops those candidates are scored exactly and the
      best k of them are the result.
"""

from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from .aps import APSParams, APSResult, CapTable, aps_search_one
from .ivf import PartitionedSet, centroid_ranking
from .knn import distances, select_topk

CODEWORDS = 256


def sub_dim(d: int, m: int) -> int:
    """Dimensions per subspace; m must divide d."""
    if m < 1 or d % m != 0:
        raise ValueError(f"{m} subspaces do not divide {d} dimensions")
    return d // m


def _sub(X: np.ndarray, s: int, ds: int) -> np.ndarray:
    return np.asarray(X, dtype=np.float64)[:, s * ds:(s + 1) * ds]


def _sq_dist(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """[len(A)][len(B)] squared Euclidean distances, written out as sums of
    squared differences."""
    diff = A[:, None, :] - B[None, :, :]
    return (diff * diff).sum(-1)


def residuals(ps: PartitionedSet) -> np.ndarray:
    """Every row of ps minus its partition's centroid (FP64)."""
    return np.asarray(ps.X, dtype=np.float64) - ps.C[ps.assign]


def train(X: np.ndarray, m: int, iters: int, seed: int) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Codebooks [m][256][d/m] (FP64) of the rows X (residuals, reading P2)
    by Lloyd's k-means in every subspace, and each subspace's distortion (mean squared error of the
    rows against their nearest codeword) before the first and after every
    iteration.  All subspaces start from the same 256 distinct rows."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    ds = sub_dim(d, m)
    if n < CODEWORDS:
        raise ValueError("training needs at least 256 rows")
    start = np.random.default_rng(seed).choice(n, CODEWORDS, replace=False)
    books = np.empty((m, CODEWORDS, ds))
    history = []
    for s in range(m):
        xs = _sub(X, s, ds)
        c = xs[start].copy()
        hist = []
        for _ in range(iters + 1):
            dist = _sq_dist(xs, c)
            a = np.argmin(dist, axis=1)
            hist.append(float(dist[np.arange(n), a].mean()))
            if len(hist) == iters + 1:
                break
            for j in range(CODEWORDS):
                members = xs[a == j]
                if members.shape[0]:
                    c[j] = members.mean(0)
        books[s] = c
        history.append(np.array(hist))
    return books, history


def encode(X: np.ndarray, books: np.ndarray, base: Optional[np.ndarray] = None) -> np.ndarray:
    """[n][m] uint8 codes of X - base (base: each row's partition centroid,
    or None for the rows themselves): the nearest codeword of every
    subspace, ties to the lower index (np.argmin keeps the first of equal
    values)."""
    X = np.asarray(X, dtype=np.float64)
    if base is not None:
        X = X - np.asarray(base, dtype=np.float64)
    m, _, ds = books.shape
    codes = np.empty((X.shape[0], m), dtype=np.uint8)
    for s in range(m):
        codes[:, s] = np.argmin(_sq_dist(_sub(X, s, ds), books[s]), axis=1)
    return codes


def decode(codes: np.ndarray, books: np.ndarray, base: Optional[np.ndarray] = None) -> np.ndarray:
    """[n][d] FP64 vectors the codes stand for (plus base when given)."""
    m, _, ds = books.shape
    out = np.empty((codes.shape[0], m * ds))
    for s in range(m):
        out[:, s * ds:(s + 1) * ds] = books[s][codes[:, s].astype(np.int64)]
    if base is not None:
        out += np.asarray(base, dtype=np.float64)
    return out


def tables(q: np.ndarray, books: np.ndarray, metric: str) -> np.ndarray:
    """[m][256] query-to-codeword values (reading P3): squared distances of
    the query's subvectors to the codewords, or their inner products."""
    m, _, ds = books.shape
    q = np.asarray(q, dtype=np.float64)
    T = np.empty((m, CODEWORDS))
    for s in range(m):
        qs = q[s * ds:(s + 1) * ds]
        if metric == "ip":
            T[s] = books[s] @ qs
        else:
            diff = books[s] - qs[None, :]
            T[s] = (diff * diff).sum(1)
    return T


def asymmetric(q: np.ndarray, codes: np.ndarray, books: np.ndarray, metric: str,
               base: Optional[np.ndarray] = None) -> np.ndarray:
    """Value of every coded row for the query (reading P3): the exact value
    of the query and the row's decoded vector (base + decoded residual)."""
    return distances(np.asarray(q)[None, :], decode(codes, books, base), metric)[0]


def rerank(q: np.ndarray, ps: PartitionedSet, ids: np.ndarray, k: int, metric: str):
    """Best k of the candidate ids by exact value (ties to the lower id)."""
    ids = np.asarray(ids, dtype=np.int64)
    ids = ids[ids >= 0]
    row_of = {int(i): r for r, i in enumerate(ps.ids.tolist())}
    rows = np.array([row_of[int(i)] for i in ids], dtype=np.int64)
    vals = distances(q[None, :], ps.X[rows], metric)[0] if rows.size else np.zeros(0)
    return select_topk(vals, ids, k, metric)


def pq_search_one(ps: PartitionedSet, codes: np.ndarray, books: np.ndarray, q: np.ndarray, params: APSParams,
                  table: CapTable, keep: int, order: Optional[np.ndarray] = None,
                  h: Optional[np.ndarray] = None):
    """APS over the compressed rows (reading P4): ``codes`` [n][m] are the
    codes of ps.X's rows' residuals to their partitions' centroids.  Returns (ids [k], values [k], the APS result over
    the scores, whose ids are the ``keep`` candidates)."""
    res: APSResult = aps_search_one(
        ps, q, params, table, order, h,
        row_values=lambda rows: asymmetric(q, codes[rows], books, params.metric, ps.C[ps.assign[rows]]), keep=keep)
    ri, rv = rerank(q, ps, res.ids, params.k, params.metric)
    return ri, rv, res


def pq_nprobe_one(ps: PartitionedSet, codes: np.ndarray, books: np.ndarray, q: np.ndarray, k: int, nprobe: int,
                  metric: str, keep: int):
    """Fixed-nprobe search over the compressed rows: the best ``keep`` rows
    of the nprobe nearest partitions by score (ties to the lower id), then
    the best k of them by exact value.  Returns (ids, values, candidates)."""
    parts = centroid_ranking(q, ps.C, metric)[1][:nprobe]
    rows = np.concatenate([ps.members[int(p)] for p in parts])
    ci, _ = select_topk(asymmetric(q, codes[rows], books, metric, ps.C[ps.assign[rows]]), ps.ids[rows], keep,
                        metric)
    ri, rv = rerank(q, ps, ci, k, metric)
    return ri, rv, ci
