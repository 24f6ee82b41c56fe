"""Comparison rules between the device's scan over product codes and the
oracle (Sec. 8, "Vector Compression"; readings P1-P4).

Tolerances (derived from the FP32 arithmetic of the device path): a code is
the nearest codeword in FP32, so another code is accepted only within 1e-5
of the residual's and codewords' squared norms; a row's score is the sum of
three FP32 terms (centroid term, residual term, table sum), each rounded
relative to its magnitude, and is bounded by 1e-5 times the sum of those
magnitudes.
"""

from __future__ import annotations

import math

import numpy as np

import parity
from oracle import knn as oknn
from oracle import pq as opq


def code_violations(X, codes, books):
    """(row, subspace) pairs whose code is not the nearest codeword beyond
    FP32 rounding of the distances."""
    m, _, ds = books.shape
    bad = []
    for s in range(m):
        sub = np.asarray(X, dtype=np.float64)[:, s * ds:(s + 1) * ds]
        dist = ((sub[:, None, :] - books[s][None]) ** 2).sum(-1)
        got = dist[np.arange(sub.shape[0]), codes[:, s].astype(np.int64)]
        best = dist.min(1)
        scale = (sub ** 2).sum(1) + (books[s] ** 2).sum(1).max()
        bad += [(int(r), s) for r in np.nonzero(got - best > 1e-5 * scale + 1e-12)[0]]
    return bad


def score_tol(q, ps, codes, books, rows, metric):
    """FP32 error bound of the device's scores of `rows`: the centroid term,
    the residual term and the table sum are each rounded, relative 1e-5 of
    their magnitudes |q - c|^2 + |r^|^2 + 2|<c, r^>| + 2|<q, r^>| (L2) or
    |<q, c>| + |<q, r^>| (IP)."""
    q64 = np.asarray(q, dtype=np.float64)
    C = ps.C[ps.assign[rows]]
    R = opq.decode(codes[rows], books)
    if metric == "ip":
        mag = np.abs(C @ q64) + np.abs(R @ q64)
    else:
        mag = ((q64 - C) ** 2).sum(1) + (R * R).sum(1) + 2 * np.abs((C * R).sum(1)) + 2 * np.abs(R @ q64)
    return 1e-5 * float(mag.max()) + 1e-6


def check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, gi, gv, where):
    """One query's device results against the oracle's scores over the
    partitions `parts`: every result is among the best kk rows by score
    (up to FP32 rounding of the scores), carries its exact value, and no row
    surely among those kk with a better exact value than the k-th result is
    missing."""
    rows = np.concatenate([ps.members[int(p)] for p in parts])
    s = opq.asymmetric(q, codes[rows], books, metric, ps.C[ps.assign[rows]])
    key = -s if metric == "ip" else s
    stol = score_tol(q, ps, codes, books, rows, metric)
    b = np.sort(key)[min(kk, key.size) - 1]
    n_res = min(k, rows.size)
    live = gi[gi >= 0]
    assert live.size == n_res, f"{where}: {live.size} results, expected {n_res}"
    assert len(set(live.tolist())) == live.size, f"{where}: repeated ids"
    pos = {int(ps.ids[r]): j for j, r in enumerate(rows)}
    assert all(int(i) in pos for i in live), f"{where}: a result outside the scanned partitions"
    rkey = np.array([key[pos[int(i)]] for i in live])
    assert (rkey <= b + stol).all(), f"{where}: a result is not among the best {kk} scores"
    id_to_row = {int(i): r for r, i in enumerate(ps.ids.tolist())}
    tv = parity.true_values(q, X, id_to_row, live, metric)
    tol = parity.value_tol(q, X, metric, tv)
    assert (np.abs(gv[:n_res] - tv) <= tol).all(), f"{where}: reported values are not the exact ones"
    ek = parity.key_of(gv[:n_res], metric)
    assert (np.diff(ek) >= 0).all(), f"{where}: results are not sorted"
    sure = rows[key < b - stol]
    if sure.size:
        ex = parity.key_of(oknn.distances(q[None], X[sure], metric)[0], metric)
        ktol = float(parity.value_tol(q, X, metric, np.array([gv[n_res - 1]]))[0])
        must = set(int(ps.ids[r]) for r, e in zip(sure, ex) if e < ek[-1] - ktol)
        assert must <= set(live.tolist()), f"{where}: missing {sorted(must - set(live.tolist()))[:5]}"


def pq_margin(res, tau, stol, upto):
    """True when a stop or recompute decision up to step `upto` is too close
    to call with scores rounded by up to stol: a recall estimate within 1e-4
    of the target, or a recompute gap |rho' - rho| - tau_rho rho within the
    rounding of the two radii (a score error of stol moves rho = sqrt(score)
    by stol / (2 rho), so the gap by up to stol / rho; IP radii the same)."""
    for st in res.steps[:upto]:
        if abs(st.recall - tau) < 1e-4:
            return True
        if math.isfinite(st.recompute_gap) and math.isfinite(st.rho_new):
            if abs(st.recompute_gap) < 2.0 * stol / max(st.rho_new, 1e-12) + 1e-5 * st.rho:
                return True
    return False
