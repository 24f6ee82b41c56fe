"""The comparison rules for the scan over product codes, checked on the CPU.

The score tolerance must cover the device's FP32 arithmetic: scores formed
as the device forms them (centroid term + residual term + table entries, in
FP32) stay within it of the FP64 values, and it is not vacuous.  The result
rules must accept the oracle's own results and reject each plausible
mistake planted in them (a row the scores did not keep, a value that is not
the exact one, a sure neighbour dropped, a broken order).
"""

import numpy as np
import pytest

import synth
from oracle import aps as oaps
from oracle import ivf as oivf
from oracle import kmeans as okm
from oracle import pq as opq
from pq_parity import check_pq_results, pq_margin, score_tol


def _setup(metric, n=6000, d=32, m=8, nlist=24):
    spec = synth.MixtureSpec(key=81, n=n, d=d, n_components=30, zipf_s=1.1, unit_norm=metric == "ip")
    X = synth.database(spec)
    Q = synth.queries(spec, 20)
    rng = np.random.default_rng(0)
    C = X[rng.choice(n, nlist, replace=False)].astype(np.float32).astype(np.float64)
    ps = oivf.PartitionedSet(X, np.arange(n, dtype=np.int64), okm.assign_nearest(X, C), C)
    books, _ = opq.train(opq.residuals(ps)[:3000], m, 3, seed=1)
    books = books.astype(np.float32).astype(np.float64)
    codes = opq.encode(ps.X, books, ps.C[ps.assign])
    return X, Q, ps, books, codes


def fp32_scores(q, ps, books, codes, rows, metric):
    """Scores as the device forms them, every operation in FP32."""
    f = np.float32
    q32 = q.astype(f)
    C32 = ps.C[ps.assign[rows]].astype(f)
    B32 = books.astype(f)
    m, _, ds = books.shape
    if metric == "ip":
        base = -(C32 * q32[None]).sum(1, dtype=f)
        key = base
    else:
        base = ((q32[None] - C32) ** 2).sum(1, dtype=f)
        R = np.concatenate([B32[s][codes[rows, s].astype(np.int64)] for s in range(m)], axis=1)
        e = (R * (R + f(2) * C32)).sum(1, dtype=f)
        key = (base + e).astype(f)
    for s in range(m):
        entry = (B32[s][codes[rows, s].astype(np.int64)] * q32[s * ds:(s + 1) * ds][None]).sum(1, dtype=f)
        key = (key + (-entry if metric == "ip" else f(-2) * entry)).astype(f)
    return key.astype(np.float64)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_score_tolerance_covers_fp32_scores(metric):
    X, Q, ps, books, codes = _setup(metric)
    rows = np.arange(X.shape[0])
    for q in Q:
        exact = opq.asymmetric(q, codes[rows], books, metric, ps.C[ps.assign[rows]])
        key = -exact if metric == "ip" else exact
        dev = fp32_scores(q, ps, books, codes, rows, metric)
        stol = score_tol(q, ps, codes, books, rows, metric)
        err = np.abs(dev - key)
        assert err.max() <= stol
        # not vacuous: far below the spread of the scores that rank the rows
        assert stol < 1e-3 * float(np.std(key))


def _oracle_result(q, ps, books, codes, metric, nprobe=4, kk=30, k=10):
    _, order = oivf.centroid_ranking(q, ps.C, metric)
    ri, rv, _ = opq.pq_nprobe_one(ps, codes, books, q, k, nprobe, metric, kk)
    return order[:nprobe], ri, rv.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_result_rules_accept_the_oracle_and_reject_planted_mistakes(metric):
    X, Q, ps, books, codes = _setup(metric)
    kk, k = 30, 10
    caught = {"outside": 0, "value": 0, "missing": 0, "order": 0}
    for i, q in enumerate(Q):
        parts, ri, rv = _oracle_result(q, ps, books, codes, metric, kk=kk, k=k)
        check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, ri, rv, f"query {i}")
        rows = np.concatenate([ps.members[int(p)] for p in parts])
        s = opq.asymmetric(q, codes[rows], books, metric, ps.C[ps.assign[rows]])
        key = -s if metric == "ip" else s
        by_score = rows[np.argsort(key, kind="stable")]
        # a row far outside the best kk scores, with its exact value, in last place
        bad_i, bad_v = ri.copy(), rv.copy()
        far = int(ps.ids[by_score[-1]])
        bad_i[-1] = far
        bad_v[-1] = float(np.float32(((X[far].astype(np.float64) - q) ** 2).sum() if metric == "l2"
                                     else X[far].astype(np.float64) @ q))
        with pytest.raises(AssertionError):
            check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, bad_i, bad_v, "planted")
        caught["outside"] += 1
        # a reported value that is not the row's exact value
        bad_v = rv.copy()
        bad_v[0] += 1e-2 * max(abs(bad_v[0]), 1.0) * (1 if metric == "l2" else -1)
        with pytest.raises(AssertionError):
            check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, ri, bad_v, "planted")
        caught["value"] += 1
        # the best result dropped for the eleventh-best exact row of the kept
        # ones (planted only where that row is surely among the kept scores)
        _, _, ci = opq.pq_nprobe_one(ps, codes, books, q, k, len(parts), metric, kk)
        alt_i, alt_v = opq.rerank(q, ps, ci, k + 1, metric)
        b = np.sort(key)[kk - 1]
        stol = score_tol(q, ps, codes, books, rows, metric)
        sure = alt_i[0] >= 0 and key[list(ps.ids[rows]).index(int(alt_i[0]))] < b - stol
        if alt_i[-1] >= 0 and sure:
            bad_i = np.concatenate([alt_i[1:k + 1]])
            bad_v = alt_v[1:k + 1].astype(np.float32).astype(np.float64)
            with pytest.raises(AssertionError):
                check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, bad_i, bad_v, "planted")
            caught["missing"] += 1
        # two results swapped
        bad_i, bad_v = ri.copy(), rv.copy()
        bad_i[[0, k - 1]] = bad_i[[k - 1, 0]]
        bad_v[[0, k - 1]] = bad_v[[k - 1, 0]]
        if bad_v[0] != bad_v[k - 1]:
            with pytest.raises(AssertionError):
                check_pq_results(q, X, ps, codes, books, parts, kk, k, metric, bad_i, bad_v, "planted")
            caught["order"] += 1
    assert min(caught.values()) >= 10, caught


def test_margin_rule():
    st = oaps.APSStep(m=3, rho=1.0, rho_new=1.2, recomputed=True, recall=0.95005, recompute_gap=0.19)
    res = oaps.APSResult(np.zeros(1, dtype=np.int64), np.zeros(1), 3, np.arange(4), np.zeros(3), [st])
    assert pq_margin(res, 0.95, 1e-6, 1)                  # the estimate is within 1e-4 of the target
    st.recall = 0.97
    assert not pq_margin(res, 0.95, 1e-6, 1)              # a clear stop and a clear recompute
    st.recompute_gap = 1e-6
    assert pq_margin(res, 0.95, 1e-6, 1)                  # the recompute is within the scores' rounding
    st.recompute_gap = 1e-2
    assert not pq_margin(res, 0.95, 1e-6, 1)
