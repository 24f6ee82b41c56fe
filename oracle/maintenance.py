"""Adaptive incremental maintenance: cost model and decision workflow (Sec. 4).

Test infrastructure only (see the package docstring).

Cost model (Sec. 4.1, Eqs. CostPartition and CostTotal): partition j of a
level contributes C_j = A_j * lambda(s_j), with A_j the fraction of queries
in the statistics window that scanned it and lambda(s) the profiled latency
of scanning s vectors; the index's cost is the sum over partitions.  An
action is judged by Delta C = C_after - C_before (Eq. DeltaC) and applied
only when Delta C < -tau.

Deltas (Sec. 4.2, "Cost Deltas"):
* exact split of j into children L, R (Eq. delta_split_exact):
  dO_plus - A_j lambda(s_j) + A_L lambda(s_L) + A_R lambda(s_R), where
  dO_plus = lambda(N + 1) - lambda(N) pays for one more centroid to scan;
* exact merge (deletion) of j into receivers m (Eq. delta_merge_exact):
  dO_minus - A_j lambda(s_j) + sum_m [(A_m + dA_m) lambda(s_m + ds_m)
  - A_m lambda(s_m)], dO_minus = lambda(N - 1) - lambda(N);
* split estimate (Eq. delta_split_est), balanced halves each inheriting a
  fraction alpha of the parent's frequency:
  dO_plus - A_j lambda(s_j) + 2 alpha A_j lambda(s_j / 2).

Workflow (Sec. 4.2, "Decision Workflow"): estimate every partition's split
(and delete) delta, tentatively apply those below -tau, verify each with the
actual sizes it produced (keeping the estimate's frequency assumptions),
commit when the verified delta is still below -tau, reject otherwise.

Readings (the paper defers the details to its technical report):
* lambda between profiled sizes is linearly interpolated, and extended
  linearly past the first and last points (the paper gives lambda only at
  sample sizes; the worked example needs it at exactly those sizes);
* verify keeps the estimate's frequency assumption for split children:
  A_L = A_R = alpha A_j;
* the merge estimate assumes uniform redistribution (its formula is
  deferred): the partition's vectors and its access frequency spread
  evenly over its r nearest receivers, ds_m = s_j / r and
  dA_m = A_j / r; at verify the receivers and their ds_m are the actual
  ones and dA_m = A_j ds_m / s_j (frequency follows the vectors).
* merge candidates: partitions below a minimum size.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np


class Latency:
    """lambda(s): piecewise-linear through profiled (size, latency) points."""

    def __init__(self, sizes: Sequence[float], values: Sequence[float]):
        s = np.asarray(sizes, dtype=np.float64)
        v = np.asarray(values, dtype=np.float64)
        order = np.argsort(s)
        self.s, self.v = s[order], v[order]
        if self.s.size < 2 or np.any(np.diff(self.s) <= 0):
            raise ValueError("need at least two distinct profiled sizes")

    def __call__(self, size: float) -> float:
        s, v = self.s, self.v
        x = float(size)
        if x <= s[0]:
            i = 0
        elif x >= s[-1]:
            i = s.size - 2
        else:
            i = int(np.searchsorted(s, x, side="right")) - 1
        t = (x - s[i]) / (s[i + 1] - s[i])
        return float(v[i] + t * (v[i + 1] - v[i]))


def partition_cost(A: float, s: float, lam: Latency) -> float:
    """C_j = A_j * lambda(s_j) (Eq. CostPartition)."""
    return float(A) * lam(s)


def total_cost(A: Sequence[float], s: Sequence[float], lam: Latency, n_centroids: Optional[int] = None) -> float:
    """Sum of the partition costs (Eq. CostTotal); with n_centroids, plus
    lambda(n_centroids), the scan of the centroids every query makes."""
    c = sum(partition_cost(a, x, lam) for a, x in zip(A, s))
    if n_centroids is not None:
        c += lam(n_centroids)
    return c


def centroid_overhead_plus(n: int, lam: Latency) -> float:
    """dO+ = lambda(N + 1) - lambda(N): one more centroid to scan."""
    return lam(n + 1) - lam(n)


def centroid_overhead_minus(n: int, lam: Latency) -> float:
    """dO- = lambda(N - 1) - lambda(N): one centroid fewer."""
    return lam(n - 1) - lam(n)


def delta_split_exact(dO_plus: float, A: float, s: float, A_L: float, s_L: float, A_R: float, s_R: float,
                      lam: Latency) -> float:
    """Eq. delta_split_exact."""
    return dO_plus - A * lam(s) + A_L * lam(s_L) + A_R * lam(s_R)


def delta_split_estimate(dO_plus: float, A: float, s: float, alpha: float, lam: Latency) -> float:
    """Eq. delta_split_est: balanced halves, each with alpha * A."""
    return dO_plus - A * lam(s) + 2.0 * alpha * A * lam(s / 2.0)


def delta_merge_exact(dO_minus: float, A: float, s: float, receivers: Sequence[Tuple[float, float, float, float]],
                      lam: Latency) -> float:
    """Eq. delta_merge_exact; receivers are (A_m, s_m, dA_m, ds_m)."""
    d = dO_minus - A * lam(s)
    for A_m, s_m, dA_m, ds_m in receivers:
        d += (A_m + dA_m) * lam(s_m + ds_m) - A_m * lam(s_m)
    return d


def delta_merge_estimate(dO_minus: float, A: float, s: float, receivers: Sequence[Tuple[float, float]],
                         lam: Latency) -> float:
    """Uniform-redistribution merge estimate (reading): receivers (A_m, s_m)
    each get s / r vectors and A / r of the frequency."""
    r = len(receivers)
    if r == 0:
        return dO_minus - A * lam(s)
    return delta_merge_exact(dO_minus, A, s, [(a, x, A / r, s / r) for a, x in receivers], lam)


@dataclass
class Decision:
    partition: int
    action: str            # "split" or "merge"
    estimate: float        # Delta' of Stage 1
    verified: float        # Delta of Stage 2 (nan when not tried)
    committed: bool


@dataclass
class SplitOutcome:
    s_L: float
    s_R: float


@dataclass
class MergeOutcome:
    receivers: List[Tuple[int, float]]   # (partition, vectors it receives)


def run_workflow(A: Sequence[float], s: Sequence[float], lam: Latency, tau: float, alpha: float,
                 dO_plus: float, split_outcome, dO_minus: float = 0.0, merge_outcome=None,
                 min_merge_size: float = 0.0, merge_receivers=None, min_split_size: float = 2.0) -> List[Decision]:
    """Stages 1-3 of the decision workflow for one level.

    dO_plus / dO_minus: the centroid-overhead terms (centroid_overhead_plus
    and _minus of the level's centroid count, or a profiled constant as in
    the worked example).  split_outcome(j) -> SplitOutcome: the sizes a
    tentative split of j actually produced.  merge_outcome(j) ->
    MergeOutcome: where a deleted j's vectors actually went.
    merge_receivers(j) -> the partitions the estimate spreads j over (the
    uniform-redistribution reading).  Every estimate is taken against the
    index as it was before the pass; a partition is tried for at most one
    action, splits first; partitions below min_split_size are not split.
    """
    A = [float(a) for a in A]
    s = [float(x) for x in s]
    out: List[Decision] = []
    taken = set()
    for j in range(len(A)):
        if s[j] < min_split_size:
            continue
        est = delta_split_estimate(dO_plus, A[j], s[j], alpha, lam)
        if est < -tau:
            o = split_outcome(j)
            ver = delta_split_exact(dO_plus, A[j], s[j], alpha * A[j], o.s_L, alpha * A[j], o.s_R, lam)
            out.append(Decision(j, "split", est, ver, ver < -tau))
            taken.add(j)
    if merge_outcome is not None:
        for j in range(len(A)):
            if j in taken or s[j] >= min_merge_size:
                continue
            rec = merge_receivers(j) if merge_receivers else []
            est = delta_merge_estimate(dO_minus, A[j], s[j], [(A[m], s[m]) for m in rec], lam)
            if est < -tau:
                o = merge_outcome(j)
                ver = delta_merge_exact(dO_minus, A[j], s[j],
                                        [(A[m], s[m], A[j] * ds / s[j] if s[j] > 0 else 0.0, ds)
                                         for m, ds in o.receivers], lam)
                out.append(Decision(j, "merge", est, ver, ver < -tau))
    return out


# ---------------------------------------------------------------- the actions on vectors
#
# Sec. 4.2 "Maintenance Actions".  Readings:
# * split: 2-means inside the partition.  Start (the paper does not fix it):
#   the row farthest from the partition's centroid, then the row farthest
#   from that one (ties to the lower row); for inner product "farthest"
#   means the smallest score and centroids are kept unit length (spherical
#   k-means, as the build).  A fixed number of Lloyd steps, then a final
#   assignment; a row equally near both goes left.  The left child keeps the
#   partition's id, the right child takes the next free id.
# * refinement: one k-means pass seeded by the current centroids over the
#   two children and the r_f nearest partitions of each child centroid
#   (union), i.e. assign every row of that group to its nearest centroid of
#   the group, recompute those centroids as means, and assign again.
# * delete (merge): every row of the partition goes to its nearest remaining
#   centroid (ties to the lower id); afterwards the surviving partitions are
#   renumbered in their old order.


def _score(X: np.ndarray, C: np.ndarray, metric: str) -> np.ndarray:
    """Ascending-is-nearer key: squared L2, or the negated inner product."""
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if metric == "ip":
        return -(X @ C.T)
    d = X[:, None, :] - C[None, :, :]
    return np.einsum("ijk,ijk->ij", d, d)


def _mean(X: np.ndarray, metric: str) -> np.ndarray:
    c = np.asarray(X, dtype=np.float64).mean(0)
    if metric == "ip":
        n = np.sqrt((c * c).sum())
        if n > 0:
            c = c / n
    return c


def _unit(c: np.ndarray, metric: str) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64)
    if metric == "ip":
        n = np.sqrt((c * c).sum())
        if n > 0:
            return c / n
    return c


def two_means(X: np.ndarray, centroid: np.ndarray, iters: int, metric: str):
    """Split rows X of one partition in two; returns (labels 0/1, [cL, cR])."""
    X = np.asarray(X, dtype=np.float64)
    far = _score(X, centroid[None, :], metric)[:, 0]
    a = int(np.argmax(far))
    far_a = _score(X, X[a][None, :], metric)[:, 0]
    b = int(np.argmax(far_a))
    C = np.stack([_unit(X[a], metric), _unit(X[b], metric)])
    for _ in range(iters):
        S = _score(X, C, metric)
        lab = (S[:, 1] < S[:, 0]).astype(np.int64)
        for c in (0, 1):
            if (lab == c).any():
                C[c] = _mean(X[lab == c], metric)
    S = _score(X, C, metric)
    lab = (S[:, 1] < S[:, 0]).astype(np.int64)
    return lab, C


def nearest_among(X: np.ndarray, C: np.ndarray, allowed: Sequence[int], metric: str) -> np.ndarray:
    """Nearest centroid id among `allowed` (ties to the lower id)."""
    allowed = np.sort(np.asarray(allowed, dtype=np.int64))
    S = _score(X, C[allowed], metric)
    return allowed[np.argmin(S, axis=1)]


def nearest_centroids(C: np.ndarray, c: np.ndarray, r: int, exclude: Sequence[int], metric: str) -> List[int]:
    """The r centroids nearest to c (ties to the lower id), skipping `exclude`."""
    key = _score(np.asarray(c, dtype=np.float64)[None, :], C, metric)[0]
    order = np.lexsort((np.arange(C.shape[0]), key))
    ex = set(int(e) for e in exclude)
    return [int(p) for p in order if int(p) not in ex][:r]


@dataclass
class MaintainParams:
    tau: float
    alpha: float
    refine_radius: int = 50
    refine_iters: int = 1
    split_iters: int = 8
    min_split_size: int = 2
    merge_below: int = 0


def maintain(X: np.ndarray, part: np.ndarray, C: np.ndarray, hits: np.ndarray, window: int, lam: Latency,
             prm: MaintainParams, metric: str):
    """One maintenance pass over a one-level index (Sec. 4.2, Stages 0-3).

    X: rows (live vectors), part: their partitions, C: centroids [N, d],
    hits[j]: queries of the window that scanned j.  Returns (part', C',
    decisions) with partitions renumbered after deletions.  The centroid
    overhead terms are taken at the partition count before the pass; every
    other quantity is read from the index as the earlier steps of the pass
    left it (split estimates need only the partition's own statistics).
    """
    X = np.asarray(X, dtype=np.float64)
    part = np.asarray(part, dtype=np.int64).copy()
    C = np.array(C, dtype=np.float64)
    N0 = C.shape[0]
    A0 = np.asarray(hits, dtype=np.float64) / float(max(window, 1))
    s0 = np.bincount(part, minlength=N0).astype(np.float64)
    dO_plus = centroid_overhead_plus(N0, lam)
    dO_minus = centroid_overhead_minus(N0, lam)
    A = list(A0)
    decisions: List[Decision] = []
    # Stage 1: estimates against the index as it stands
    split_est = {j: delta_split_estimate(dO_plus, A0[j], s0[j], prm.alpha, lam) for j in range(N0)
                 if s0[j] >= prm.min_split_size}
    # Stages 2-3 for splits, in partition order
    committed_splits = []
    for j in range(N0):
        est = split_est.get(j)
        if est is None or not est < -prm.tau:
            continue
        rows = np.nonzero(part == j)[0]
        lab, CC = two_means(X[rows], C[j], prm.split_iters, metric)
        sL, sR = float((lab == 0).sum()), float((lab == 1).sum())
        ver = delta_split_exact(dO_plus, A0[j], s0[j], prm.alpha * A0[j], sL, prm.alpha * A0[j], sR, lam)
        ok = ver < -prm.tau
        decisions.append(Decision(j, "split", est, ver, ok))
        if ok:
            r = C.shape[0]
            C = np.vstack([C, CC[1][None, :]])
            C[j] = CC[0]
            part[rows[lab == 1]] = r
            A[j] = prm.alpha * A0[j]
            A.append(prm.alpha * A0[j])
            committed_splits.append((j, r))
    # refinement around each committed split, in commit order
    for j, r in committed_splits:
        if prm.refine_iters <= 0:
            continue
        group = {j, r}
        for c in (j, r):
            group.update(nearest_centroids(C, C[c], prm.refine_radius, exclude=(j, r), metric=metric))
        group = sorted(group)
        rows = np.nonzero(np.isin(part, group))[0]
        for _ in range(prm.refine_iters):
            lab = nearest_among(X[rows], C, group, metric)
            for g in group:
                sel = lab == g
                if sel.any():
                    C[g] = _mean(X[rows[sel]], metric)
        part[rows] = nearest_among(X[rows], C, group, metric)
    # deletes, in partition order, estimated and verified against the index
    # as the splits and earlier deletes of this pass left it
    split_parts = set(j for j, _ in committed_splits) | set(d.partition for d in decisions)
    deleted = []
    if prm.merge_below > 0:
        for j in range(N0):
            rows = np.nonzero(part == j)[0]
            sj = float(rows.size)
            if j in split_parts or not sj < prm.merge_below:
                continue
            alive = [p for p in range(C.shape[0]) if p != j and p not in deleted]
            if not alive:
                continue
            rec = nearest_centroids(C, C[j], prm.refine_radius, exclude=[j] + deleted, metric=metric)
            est = delta_merge_estimate(dO_minus, A0[j], sj, [(A[m], float((part == m).sum())) for m in rec], lam)
            if not est < -prm.tau:
                continue
            dest = nearest_among(X[rows], C, alive, metric) if rows.size else np.zeros(0, dtype=np.int64)
            recv = []
            for m in np.unique(dest):
                ds = float((dest == m).sum())
                recv.append((A[m], float((part == m).sum()), A0[j] * ds / sj, ds))
            ver = delta_merge_exact(dO_minus, A0[j], sj, recv, lam)
            ok = ver < -prm.tau
            decisions.append(Decision(j, "merge", est, ver, ok))
            if ok:
                part[rows] = dest
                deleted.append(j)
    if deleted:
        keep = [p for p in range(C.shape[0]) if p not in deleted]
        remap = -np.ones(C.shape[0], dtype=np.int64)
        remap[keep] = np.arange(len(keep))
        C = C[keep]
        part = remap[part]
    return part, C, decisions
