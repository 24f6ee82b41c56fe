"""Adaptive Partition Scanning, one index level (Sec. 5).

Test infrastructure only (see the package docstring).

Geometric model (Sec. 5, "Geometric Model", Eq. aps-pi): with rho the distance from the query
to its k-th nearest neighbour found so far, the chance that partition P_i
holds a neighbour is the share of the ball B(q, rho) inside P_i.  Each
neighbouring partition is approximated by the half-space beyond the
bisector of the query's nearest centroid c_0 and c_i; the share of the ball
beyond a hyperplane at distance h from q is a hyperspherical cap whose
volume fraction, for t = h / rho in [0, 1), is

    v(t) = 1/2 * I_{1 - t^2}((d + 1) / 2, 1/2)

(regularised incomplete beta function; the closed form the paper cites in
the same paragraph).  v(t) = 0 for t >= 1.

Nearest-partition probability (Eq. aps-p0) and the split of the rest
(Eq. aps-pi-final): p_0 = prod_j (1 - v_j); p_i = (1 - p_0) * v_i / sum_j v_j.

Readings of points the paper leaves open (each is also listed with its
reason in the design notes):
* R1  p_0 takes the raw cap fractions; only the split of 1 - p_0 uses the
      normalised ones.  (Read literally, normalising first makes p_0 depend
      on the number of candidates only.)
* R2  the 1,024-point precomputed table is indexed by t = h / rho on an
      even grid t_j = j / 1023, j = 0..1023, with linear interpolation
      (Sec. 5.1, "Performance Optimizations").
* R3  until k results exist rho = +inf, every t = 0, and the estimated
      recall is held at 0.
* R4  the recompute test compares against the rho of the last recompute;
      the first finite rho always triggers one.
* R5  M = ceil(f_M * N_l) candidates, clamped to [1, N_l]; the product
      f_M * N_l is taken with a 1e-9 allowance so that 0.05 * 1000 gives 50.
* R6  inner product: the bisector of c_0 and c_i is the boundary of their
      inner-product cells, so h_i = q.(c_0 - c_i) / |c_0 - c_i|; rho is the
      Euclidean distance implied by the k-th score for unit-norm data,
      sqrt(max(0, |q|^2 + 1 - 2 s_k)).
* R7  beta parameters a = (d + 1) / 2, b = 1/2.
* Candidate order: "largest p_i first" equals ascending h (all caps share
  one rho and v is decreasing in t); ties by centroid value, then id.

Filters (Sec. 8, "Filters": the paper names the idea only):
* F1  a candidate's cap share v_i becomes the share of passing rows beyond
      its bisector, u_i = v_i f_i / (v_i f_i + (1 - v_i) f_0), with f_i the
      estimated pass fraction of P_i and f_0 that of P_0; p_0 and p_i then
      follow Eqs. aps-p0 and aps-pi-final with u in place of v.
* F2  a row passes when its 32 label bits share a bit with the query's
      mask; f_i sums the per-bit counts of the mask's bits (exact for one
      label per row), capped at the partition's live rows.

Estimator variants (Sec. 5.1, Table tab:recall_overhead): APS recomputes
p_0 and p_i only when rho moved by more than tau_rho and reads the cap
share from the table; APS-R recomputes after every partition, still from
the table; APS-RP recomputes after every partition and evaluates the cap
share directly (``ExactCap``).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
from scipy.special import betainc

from .ivf import PartitionedSet
from .knn import distances, merge_topk, select_topk, sort_key

TABLE_POINTS = 1024


def candidate_count(f_M: float, n_list: int) -> int:
    """M = ceil(f_M * N_l), clamped to [1, N_l] (reading R5)."""
    m = int(math.ceil(f_M * n_list - 1e-9))
    return max(1, min(n_list, m))


def cap_fraction(t, d: int):
    """Volume share of a d-ball beyond a hyperplane at distance t (ball radius 1)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    inside = t < 1.0
    tt = np.abs(t[inside])
    half = 0.5 * betainc((d + 1) / 2.0, 0.5, 1.0 - tt * tt)
    out[inside] = np.where(t[inside] >= 0, half, 1.0 - half)
    return out


class ExactCap:
    """cap_fraction evaluated directly at every call, with no table: the
    estimator of the variant that recomputes without precomputation
    (APS-RP, Sec. 5.1 and Table tab:recall_overhead).  Negative t is taken
    as 0, as the table does."""

    def __init__(self, d: int):
        self.d = d

    def __call__(self, t: np.ndarray) -> np.ndarray:
        return cap_fraction(np.maximum(np.asarray(t, dtype=np.float64), 0.0), self.d)


class CapTable:
    """cap_fraction sampled at TABLE_POINTS even points of t in [0, 1] (R2)."""

    def __init__(self, d: int, points: int = TABLE_POINTS):
        self.d = d
        self.points = points
        self.grid = np.linspace(0.0, 1.0, points)
        self.values = cap_fraction(self.grid, d)

    def __call__(self, t: np.ndarray) -> np.ndarray:
        t = np.asarray(t, dtype=np.float64)
        out = np.zeros_like(t)
        ok = t < 1.0
        pos = np.maximum(t[ok], 0.0) * (self.points - 1)
        j = np.minimum(np.floor(pos).astype(np.int64), self.points - 2)
        frac = pos - j
        out[ok] = self.values[j] + frac * (self.values[j + 1] - self.values[j])
        return out


@dataclass
class APSParams:
    k: int
    recall_target: float
    f_M: float = 0.05
    tau_rho: float = 0.01
    metric: str = "l2"
    # recompute p_0 and p_i after every partition scanned, whatever rho did
    # (the APS-R and APS-RP variants of Table tab:recall_overhead); otherwise
    # only when rho moved by more than tau_rho * rho
    recompute_every: bool = False


@dataclass
class APSStep:
    m: int            # partitions scanned so far
    rho: float        # rho in use after this step
    rho_new: float    # k-th distance after this step
    recomputed: bool
    recall: float     # estimate r after this step
    recompute_gap: float  # |rho' - rho| - tau_rho * rho (inf when rho was inf or every step recomputes)


@dataclass
class APSResult:
    ids: np.ndarray
    vals: np.ndarray
    m: int
    order: np.ndarray          # candidate partitions in scan order (c_0 first)
    h: np.ndarray              # bisector distances of order[1:]
    steps: List[APSStep] = field(default_factory=list)


def euclid_radius(kth_val: float, q_norm2: float, metric: str) -> float:
    """Euclidean distance to the k-th result (R6 for inner product)."""
    if not np.isfinite(kth_val):
        return math.inf
    if metric == "ip":
        return math.sqrt(max(0.0, q_norm2 + 1.0 - 2.0 * kth_val))
    return math.sqrt(max(0.0, kth_val))


def bisector_distances(q: np.ndarray, C: np.ndarray, vals: np.ndarray, c0: int, others: np.ndarray,
                       metric: str) -> np.ndarray:
    """h_i for every i in ``others`` (FP64).

    L2: (D_i^2 - D_0^2) / (2 |c_i - c_0|) from the squared distances D^2.
    IP: (s_0 - s_i) / |c_0 - c_i| from the scores s.
    A zero centroid separation gives h = 0.
    """
    C64 = np.asarray(C, dtype=np.float64)
    sep = np.sqrt(((C64[others] - C64[c0]) ** 2).sum(1))
    if metric == "ip":
        num = vals[c0] - vals[others]
    else:
        num = (vals[others] - vals[c0]) / 2.0
    h = np.zeros(others.shape[0])
    nz = sep > 0
    h[nz] = num[nz] / sep[nz]
    return h


def aps_order(q: np.ndarray, C: np.ndarray, f_M: float, metric: str, cands: Optional[np.ndarray] = None):
    """Candidate set S, c_0 and the scan order by ascending h.

    S is the M nearest centroids (Alg. "Adaptive Partition Scanning"), or,
    when ``cands`` is given (the level above returned them), all of those.
    """
    N = C.shape[0]
    vals = distances(q[None, :], C, metric)[0]
    key = sort_key(vals, metric)
    if cands is None:
        by_value = np.lexsort((np.arange(N), key))
        M = candidate_count(f_M, N)
        S = by_value[:M]
    else:
        cands = np.asarray(cands, dtype=np.int64)
        S = cands[np.lexsort((cands, key[cands]))]
    c0 = int(S[0])
    others = S[1:]
    h = bisector_distances(q, C, vals, c0, others, metric)
    o = np.lexsort((others, key[others], h))
    return np.concatenate([[c0], others[o]]).astype(np.int64), h[o]


def pass_fractions(ps: PartitionedSet, attr: np.ndarray, mask: int) -> np.ndarray:
    """Estimated share of each partition's rows that pass a filter (Sec. 8,
    "Filters"): a row passes when its label bits share a bit with `mask`; the
    estimate counts the rows carrying each bit of the mask and sums the
    counts (exact when every row carries one bit, an upper bound otherwise),
    capped at the partition's size.  Empty partitions get 0."""
    attr = np.asarray(attr, dtype=np.uint64)
    bits = [b for b in range(32) if (int(mask) >> b) & 1]
    f = np.zeros(ps.nlist)
    for p in range(ps.nlist):
        rows = ps.members[p]
        if rows.shape[0] == 0:
            continue
        a = attr[rows]
        est = sum(int(((a >> np.uint64(b)) & np.uint64(1)).sum()) for b in bits)
        f[p] = min(rows.shape[0], est) / rows.shape[0]
    return f


def filtered_share(v: np.ndarray, f: np.ndarray, f0: float) -> np.ndarray:
    """Cap shares scaled for a filter (reading F1): of the passing rows in the
    ball, the share beyond the bisector of c_0 and c_i when the rows beyond it
    pass with fraction f_i and those on c_0's side with f_0,
        u_i = v_i f_i / (v_i f_i + (1 - v_i) f_0),
    and 0 where v_i f_i = 0.  With equal fractions u_i = v_i."""
    num = v * f
    den = num + (1.0 - v) * f0
    return np.where(num > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)


class _Estimator:
    """p_0 and p_i for the current rho (Eqs. aps-p0 and aps-pi-final, reading R1),
    with the cap shares scaled by pass fractions under a filter (reading F1)."""

    def __init__(self, h: np.ndarray, table: CapTable, f: Optional[np.ndarray] = None, f0: float = 1.0):
        self.h = h
        self.table = table
        self.f = f
        self.f0 = f0
        self.p0 = 1.0
        self.p = np.zeros(h.shape[0])

    def recompute(self, rho: float):
        t = np.zeros_like(self.h) if math.isinf(rho) else self.h / rho
        v = self.table(t)
        if self.f is not None:
            v = filtered_share(v, self.f, self.f0)
        V = float(v.sum())
        self.p0 = float(np.prod(1.0 - v))
        if V > 0.0:
            self.p = (1.0 - self.p0) * v / V
        else:
            self.p0 = 1.0
            self.p = np.zeros_like(v)

    def recall(self, scanned_after_c0: int) -> float:
        return self.p0 + float(self.p[:scanned_after_c0].sum())


def aps_search_one(ps: PartitionedSet, q: np.ndarray, params: APSParams, table: CapTable,
                   order: Optional[np.ndarray] = None, h: Optional[np.ndarray] = None,
                   attr: Optional[np.ndarray] = None, mask: Optional[int] = None,
                   row_values: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                   keep: Optional[int] = None) -> APSResult:
    """Algorithm "Adaptive Partition Scanning" for one query.

    ``order``/``h`` may be given to replay a specific candidate order; by
    default they come from :func:`aps_order`.  With ``attr`` (label bits of
    every row) and ``mask``, only rows sharing a bit with the mask are
    results, and the recall model scales its cap shares by each candidate's
    pass fraction (Sec. 8, "Filters"; readings F1, F2).

    ``row_values(rows)`` replaces the exact values of the scanned rows (a
    compressed scan's scores, Sec. 8, "Vector Compression"), and the result
    list keeps the best ``keep`` >= k rows by them; rho still comes from the
    k-th value of that list.
    """
    metric = params.metric
    k = params.k
    keep = k if keep is None else int(keep)
    assert keep >= k
    if order is None:
        order, h = aps_order(q, ps.C, params.f_M, metric)
    q64 = np.asarray(q, dtype=np.float64)
    qn2 = float(q64 @ q64)

    filt = attr is not None and mask is not None
    if filt:
        attr64 = np.asarray(attr, dtype=np.uint64)

    def scan(p):
        rows = ps.members[int(p)]
        if filt:
            rows = rows[(attr64[rows] & np.uint64(int(mask))) != 0]
        if rows.shape[0] == 0:
            return select_topk(np.zeros(0), np.zeros(0, dtype=np.int64), keep, metric)
        vals = distances(q[None, :], ps.X[rows], metric)[0] if row_values is None else row_values(rows)
        return select_topk(vals, ps.ids[rows], keep, metric)

    def kth_radius(ids, vals):
        if ids[k - 1] < 0:
            return math.inf
        return euclid_radius(float(vals[k - 1]), qn2, metric)

    # Scan P_0 and set rho.
    res_i, res_v = scan(order[0])
    m = 1
    rho = kth_radius(res_i, res_v)
    if filt:
        frac = pass_fractions(ps, attr, mask)
        est = _Estimator(np.asarray(h, dtype=np.float64), table, frac[np.asarray(order[1:], dtype=np.int64)],
                         float(frac[int(order[0])]))
    else:
        est = _Estimator(np.asarray(h, dtype=np.float64), table)
    est.recompute(rho)
    full = res_i[k - 1] >= 0
    r = est.recall(0) if full else 0.0
    steps = [APSStep(m, rho, rho, True, r, math.inf)]
    M = order.shape[0]
    while r < params.recall_target and m < M:
        ti, tv = scan(order[m])
        res_i, res_v = merge_topk(res_i, res_v, ti, tv, keep, metric)
        m += 1
        rho_new = kth_radius(res_i, res_v)
        if params.recompute_every:
            gap = math.inf
            do = True
        elif math.isinf(rho):
            gap = math.inf
            do = not math.isinf(rho_new)
        else:
            gap = abs(rho_new - rho) - params.tau_rho * rho
            do = gap > 0.0
        if do:
            rho = rho_new
            est.recompute(rho)
        full = res_i[k - 1] >= 0
        r = est.recall(m - 1) if full else 0.0
        steps.append(APSStep(m, rho, rho_new, do, r, gap))
    return APSResult(res_i, res_v, m, order, np.asarray(h), steps)


def aps_search(ps: PartitionedSet, Q: np.ndarray, params: APSParams, table: Optional[CapTable] = None,
               orders=None, attr: Optional[np.ndarray] = None, masks: Optional[np.ndarray] = None):
    """APS for every query: (ids [nq,k], values [nq,k], m [nq], per-query results).
    With ``attr`` and ``masks`` (one per query) the searches are filtered."""
    table = table or CapTable(ps.X.shape[1])
    nq = Q.shape[0]
    out_i = np.empty((nq, params.k), dtype=np.int64)
    out_v = np.empty((nq, params.k))
    ms = np.empty(nq, dtype=np.int64)
    results = []
    for i in range(nq):
        o, h = (None, None) if orders is None else orders[i]
        res = aps_search_one(ps, Q[i], params, table, o, h, attr, None if masks is None else int(masks[i]))
        out_i[i], out_v[i], ms[i] = res.ids, res.vals, res.m
        results.append(res)
    return out_i, out_v, ms, results
