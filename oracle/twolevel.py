"""Search through a two-level (or deeper) partitioned index (Sec. 3 and Sec. 5).

Test infrastructure only (see the package docstring).

Level 0 partitions the vectors; level 1 partitions the level-0 centroids;
the top is one partition (Sec. 3).  APS runs at each level independently
(Sec. 5), with the upper level's recall target fixed high (99% in the
paper, Sec. 5.1 and Table two_level_results) and its own candidate
fraction (25% at level 1, 1.5% at level 0 in the paper's Sift10M runs).

Reading (the paper does not spell out the hand-over between levels): the
upper level is a k-NN search over the level-0 centroids with
k_1 = M_0 = ceil(f_M(0) * N_0); the centroids it returns, in (distance, id)
order, are the level-0 candidate set S, and c_0 is the nearest of them.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .aps import APSParams, CapTable, aps_order, aps_search_one, candidate_count
from .ivf import PartitionedSet


@dataclass
class TwoLevelParams:
    k: int
    recall_target: float
    f_M: float = 0.015
    upper_recall_target: float = 0.99
    upper_f_M: float = 0.25
    tau_rho: float = 0.01
    metric: str = "l2"


class TwoLevelSet:
    """Level 0: vectors in leaves; level 1: leaf centroids in top partitions."""

    def __init__(self, leaves: PartitionedSet, top_assign: np.ndarray, top_centroids: np.ndarray):
        self.leaves = leaves
        n0 = leaves.nlist
        self.top = PartitionedSet(leaves.C, np.arange(n0, dtype=np.int64), top_assign, top_centroids)


def two_level_search_one(tl: TwoLevelSet, q: np.ndarray, p: TwoLevelParams, table: CapTable):
    n0 = tl.leaves.nlist
    m0 = candidate_count(p.f_M, n0)
    upper = APSParams(k=m0, recall_target=p.upper_recall_target, f_M=p.upper_f_M,
                      tau_rho=p.tau_rho, metric=p.metric)
    r1 = aps_search_one(tl.top, q, upper, table)
    cands = r1.ids[r1.ids >= 0]
    order, h = aps_order(q, tl.leaves.C, p.f_M, p.metric, cands=cands)
    lower = APSParams(k=p.k, recall_target=p.recall_target, f_M=p.f_M, tau_rho=p.tau_rho, metric=p.metric)
    r0 = aps_search_one(tl.leaves, q, lower, table, order=order, h=h)
    return r0, r1


def two_level_search(tl: TwoLevelSet, Q: np.ndarray, p: TwoLevelParams, table: CapTable = None):
    table = table or CapTable(tl.leaves.X.shape[1])
    nq = Q.shape[0]
    ids = np.empty((nq, p.k), dtype=np.int64)
    vals = np.empty((nq, p.k))
    m0 = np.empty(nq, dtype=np.int64)
    m1 = np.empty(nq, dtype=np.int64)
    for i in range(nq):
        r0, r1 = two_level_search_one(tl, Q[i], p, table)
        ids[i], vals[i], m0[i], m1[i] = r0.ids, r0.vals, r0.m, r1.m
    return ids, vals, m0, m1


class LevelStack:
    """Level 0 partitions the vectors; every level l >= 1 partitions the
    centroids of level l - 1 (Sec. 3).  ``uppers`` lists (assign, centroids)
    of levels 1, 2, ... from the bottom up."""

    def __init__(self, leaves: PartitionedSet, uppers):
        self.levels = [leaves]
        for assign, C in uppers:
            below = self.levels[-1]
            self.levels.append(PartitionedSet(below.C, np.arange(below.nlist, dtype=np.int64), assign, C))


def multi_level_search_one(ls: LevelStack, q: np.ndarray, p: TwoLevelParams, table: CapTable):
    """APS at every level from the top down (Sec. 3, Sec. 5), extending the
    two-level hand-over: the search at level l >= 1 is a k-NN search over the
    centroids of level l - 1 with k_l = M_{l-1} = ceil(f_M(l-1) N_{l-1})
    (f_M(0) = p.f_M, the upper fraction above), at the upper recall target;
    its results, nearest first, are the candidate set of the search below.
    Only the top level takes its candidates from all of its centroids.
    Returns the level-0 result and the upper results from the top down."""
    uppers = []
    cands = None
    for l in range(len(ls.levels) - 1, 0, -1):
        below = ls.levels[l - 1]
        k_l = candidate_count(p.f_M if l == 1 else p.upper_f_M, below.nlist)
        prm = APSParams(k=k_l, recall_target=p.upper_recall_target, f_M=p.upper_f_M, tau_rho=p.tau_rho,
                        metric=p.metric)
        if cands is None:
            r = aps_search_one(ls.levels[l], q, prm, table)
        else:
            order, h = aps_order(q, ls.levels[l].C, p.upper_f_M, p.metric, cands=cands)
            r = aps_search_one(ls.levels[l], q, prm, table, order=order, h=h)
        uppers.append(r)
        cands = r.ids[r.ids >= 0]
    lower = APSParams(k=p.k, recall_target=p.recall_target, f_M=p.f_M, tau_rho=p.tau_rho, metric=p.metric)
    if cands is None:
        return aps_search_one(ls.levels[0], q, lower, table), uppers
    order, h = aps_order(q, ls.levels[0].C, p.f_M, p.metric, cands=cands)
    return aps_search_one(ls.levels[0], q, lower, table, order=order, h=h), uppers

