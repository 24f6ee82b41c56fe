"""Pins for the recall model and Adaptive Partition Scanning in the oracle.

The cap-volume function is checked against elementary closed forms (1-, 2-
and 3-balls, stored in tests/golden) and Monte Carlo; the table against the
library beta function; the algorithm against exact search (f_M = 1,
target 1), against a 2-D trace whose every number follows from the disc
formula, and against invariants that any correct implementation keeps.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import aps, ivf, knn, kmeans, twolevel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def disc_cap(t):
    """Share of a unit disc beyond a chord at distance t (elementary geometry)."""
    return (math.acos(t) - t * math.sqrt(1.0 - t * t)) / math.pi


def test_cap_fraction_closed_forms():
    g = json.load(open(os.path.join(GOLDEN, "cap_fraction_closed_forms.json")))
    for c in g["cases"]:
        got = float(aps.cap_fraction(np.array([c["t"]]), c["n"])[0])
        assert abs(got - c["value"]) < 1e-14, c


def test_cap_fraction_general_closed_forms():
    ts = np.linspace(0, 0.999, 57)
    np.testing.assert_allclose(aps.cap_fraction(ts, 1), 0.5 * (1 - ts), atol=1e-14)
    np.testing.assert_allclose(aps.cap_fraction(ts, 2), [disc_cap(t) for t in ts], atol=1e-14)
    np.testing.assert_allclose(aps.cap_fraction(ts, 3), (1 - ts) ** 2 * (2 + ts) / 4, atol=1e-14)
    assert aps.cap_fraction(np.array([1.0, 1.5]), 64).tolist() == [0.0, 0.0]


@pytest.mark.parametrize("n,t", [(8, 0.3), (128, 0.05), (768, 0.02)])
def test_cap_fraction_monte_carlo(n, t):
    rng = np.random.default_rng(n)
    samples = 200_000
    hits = 0
    for _ in range(4):
        g = rng.standard_normal((samples // 4, n))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        r = rng.random(samples // 4) ** (1.0 / n)
        hits += int(((g[:, 0] * r) > t).sum())
    frac = hits / samples
    exp = float(aps.cap_fraction(np.array([t]), n)[0])
    sigma = math.sqrt(exp * (1 - exp) / samples)
    assert abs(frac - exp) < 5 * sigma


@pytest.mark.parametrize("d", [2, 128, 768])
def test_table_interpolation_error(d):
    tab = aps.CapTable(d)
    ts = np.random.default_rng(0).random(5000)
    err = np.abs(tab(ts) - aps.cap_fraction(ts, d)).max()
    assert err < 3e-5
    assert tab(np.array([1.0, 2.0])).tolist() == [0.0, 0.0]
    assert abs(tab(np.array([0.0]))[0] - 0.5) < 1e-15


def test_candidate_count():
    assert aps.candidate_count(0.05, 1000) == 50
    assert aps.candidate_count(0.05, 256) == 13
    assert aps.candidate_count(0.015, 50_000) == 750
    assert aps.candidate_count(0.05, 4096) == 205
    assert aps.candidate_count(1e-9, 100) == 1
    assert aps.candidate_count(2.0, 100) == 100


def test_bisector_distance_geometry():
    C = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 4.0]])
    q = np.array([0.25, 0.5])
    vals = knn.distances(q[None], C, "l2")[0]
    h = aps.bisector_distances(q, C, vals, 0, np.array([1, 2]), "l2")
    np.testing.assert_allclose(h, [0.75, 1.5], rtol=1e-14)
    # inner product with unit centroids: the cell boundary of c0, c1 is the
    # line through the origin at 45 degrees; q = (1, 0.2) lies 0.8/sqrt(2) from it
    Cu = np.array([[1.0, 0.0], [0.0, 1.0]])
    q = np.array([1.0, 0.2])
    vals = knn.distances(q[None], Cu, "ip")[0]
    h = aps.bisector_distances(q, Cu, vals, 0, np.array([1]), "ip")
    np.testing.assert_allclose(h, [0.8 / math.sqrt(2)], rtol=1e-14)


def _two_d_index(p0_point):
    C = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 4.0]], dtype=np.float32)
    X = np.array([p0_point, [1.05, 0.5], [0.25, 2.4]], dtype=np.float32)
    assign = np.array([0, 1, 2])
    assert (kmeans.assign_nearest(X, C) == assign).all()
    return ivf.PartitionedSet(X, np.array([100, 101, 102]), assign, C)


def test_aps_trace_two_d_without_recompute():
    # q is 0.8 from the P0 point; bisector of c0,c1 is x = 1 (h = 0.75),
    # of c0,c2 is y = 2 (h = 1.5 > rho, so its cap is empty).
    ps = _two_d_index([0.25, -0.3])
    q = np.array([0.25, 0.5], dtype=np.float32)
    tab = aps.CapTable(2)
    v1 = disc_cap(0.75 / 0.8)
    res = aps.aps_search_one(ps, q, aps.APSParams(k=1, recall_target=0.99, f_M=1.0, metric="l2"), tab)
    assert res.order.tolist() == [0, 1, 2]
    assert res.m == 1 and res.ids.tolist() == [100]
    assert abs(res.steps[0].recall - (1 - v1)) < 1e-5
    res = aps.aps_search_one(ps, q, aps.APSParams(k=1, recall_target=0.995, f_M=1.0, metric="l2"), tab)
    assert res.m == 2 and not res.steps[1].recomputed
    assert abs(res.steps[1].recall - 1.0) < 1e-12


def test_aps_trace_two_d_with_recompute():
    ps = _two_d_index([0.25, -0.7])          # rho after P0 = 1.2
    q = np.array([0.25, 0.5], dtype=np.float32)
    tab = aps.CapTable(2)
    res = aps.aps_search_one(ps, q, aps.APSParams(k=1, recall_target=0.9, f_M=1.0, metric="l2"), tab)
    v_first = disc_cap(0.75 / 1.2)
    assert abs(res.steps[0].recall - (1 - v_first)) < 1e-5
    # P1's point at distance 0.8 becomes the neighbour; rho shrinks by a third,
    # the model is recomputed, and with everything of positive mass scanned r = 1
    assert res.m == 2 and res.steps[1].recomputed
    assert abs(res.steps[1].rho - 0.8) < 1e-6
    assert res.ids.tolist() == [101]
    assert abs(res.steps[1].recall - 1.0) < 1e-12


def test_probabilities_sum_to_one():
    rng = np.random.default_rng(2)
    tab = aps.CapTable(16)
    for _ in range(50):
        h = rng.random(rng.integers(1, 40)) * 2
        est = aps._Estimator(h, tab)
        est.recompute(float(rng.random() + 0.1))
        assert abs(est.p0 + est.p.sum() - 1.0) < 1e-12
        assert est.recall(h.shape[0]) == pytest.approx(1.0, abs=1e-12)


def _mixture_index(metric, n=6000, d=8, comps=20, nlist=48, seed=3):
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((comps, d)) * 2
    X = (mu[rng.integers(0, comps, n)] + 0.5 * rng.standard_normal((n, d))).astype(np.float32)
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    C0 = X[rng.choice(n, nlist, replace=False)]
    C, a, _ = kmeans.lloyd(X, C0, 5)
    C = C.astype(np.float32)
    if metric == "ip":
        C /= np.linalg.norm(C, axis=1, keepdims=True)
        a = np.argmax(X.astype(np.float64) @ C.T.astype(np.float64), 1)
    else:
        a = kmeans.assign_nearest(X, C)
    Q = (X[rng.choice(n, 40, replace=False)] + 0.1 * rng.standard_normal((40, d))).astype(np.float32)
    if metric == "ip":
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return ivf.PartitionedSet(X, np.arange(n), a, C), Q


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_full_scan_target_one_is_exact(metric):
    ps, Q = _mixture_index(metric)
    p = aps.APSParams(k=10, recall_target=1.0, f_M=1.0, metric=metric)
    gi, gv, ms, _ = aps.aps_search(ps, Q, p)
    ei, ev = knn.knn_exact(ps.X, ps.ids, Q, 10, metric)
    assert (gi == ei).all()


def test_m_non_decreasing_in_target():
    ps, Q = _mixture_index("l2")
    prev = None
    for tau in (0.5, 0.8, 0.9, 0.95, 0.99):
        _, _, ms, _ = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=tau, f_M=0.25))
        if prev is not None:
            assert (ms >= prev).all()
        prev = ms


def test_single_candidate_stops_after_p0():
    ps, Q = _mixture_index("l2")
    _, _, ms, res = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=0.999, f_M=1e-6))
    assert (ms == 1).all()
    assert all(r.steps[0].recall == 1.0 for r in res)


def test_recall_held_at_zero_until_k_results():
    C = np.array([[0.0, 0.0], [3.0, 0.0]], dtype=np.float32)
    X = np.array([[0.1, 0.0], [3.1, 0.0], [3.2, 0.0]], dtype=np.float32)
    ps = ivf.PartitionedSet(X, np.arange(3), np.array([0, 1, 1]), C)
    res = aps.aps_search_one(ps, np.zeros(2, np.float32), aps.APSParams(k=2, recall_target=0.5, f_M=1.0),
                             aps.CapTable(2))
    assert res.steps[0].recall == 0.0 and math.isinf(res.steps[0].rho)
    assert res.m == 2 and res.steps[1].recomputed
    assert res.ids.tolist() == [0, 1]


@pytest.mark.parametrize("tau", [0.8, 0.9])
def test_calibration_band(tau):
    """Achieved recall tracks the target (the paper reports a slight overshoot)."""
    ps, Q = _mixture_index("l2", n=20000, d=16, comps=40, nlist=100, seed=8)
    truth, _ = knn.knn_exact(ps.X, ps.ids, Q, 10, "l2")
    gi, _, _, _ = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=tau, f_M=0.2))
    rec = knn.recall_at_k(gi, truth, 10).mean()
    assert rec >= tau - 0.02


def test_two_level_full_upper_equals_single_level():
    ps, Q = _mixture_index("l2", n=8000, nlist=64)
    rng = np.random.default_rng(1)
    C1, a1, _ = kmeans.lloyd(ps.C, ps.C[rng.choice(64, 6, replace=False)], 4)
    a1 = kmeans.assign_nearest(ps.C, C1)
    tl = twolevel.TwoLevelSet(ps, a1, C1.astype(np.float32))
    p = twolevel.TwoLevelParams(k=10, recall_target=0.9, f_M=0.2, upper_recall_target=1.0, upper_f_M=1.0)
    gi, _, m0, _ = twolevel.two_level_search(tl, Q, p)
    si, _, sm, _ = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=0.9, f_M=0.2))
    assert (gi == si).all() and (m0 == sm).all()


def _three_levels():
    ps, Q = _mixture_index("l2", n=8000, nlist=64)
    rng = np.random.default_rng(2)
    C1, _, _ = kmeans.lloyd(ps.C, ps.C[rng.choice(64, 12, replace=False)], 4)
    a1 = kmeans.assign_nearest(ps.C, C1)
    C2, _, _ = kmeans.lloyd(C1, C1[rng.choice(12, 3, replace=False)], 4)
    a2 = kmeans.assign_nearest(C1, C2)
    return ps, Q, (a1, C1.astype(np.float32)), (a2, C2.astype(np.float32))


def test_multi_level_search_of_two_levels_is_the_two_level_search():
    ps, Q, l1, _ = _three_levels()
    tl = twolevel.TwoLevelSet(ps, l1[0], l1[1])
    ls = twolevel.LevelStack(ps, [l1])
    tab = aps.CapTable(ps.X.shape[1])
    p = twolevel.TwoLevelParams(k=10, recall_target=0.9, f_M=0.2, upper_recall_target=0.99, upper_f_M=0.5)
    for q in Q:
        r0, r1 = twolevel.two_level_search_one(tl, q, p, tab)
        m0, ups = twolevel.multi_level_search_one(ls, q, p, tab)
        assert m0.ids.tolist() == r0.ids.tolist() and m0.m == r0.m
        assert len(ups) == 1 and ups[0].ids.tolist() == r1.ids.tolist()


def test_three_levels_with_exact_upper_levels_equal_one_level():
    """Scanning every upper partition to recall 1 makes every upper search
    exact, so the level-0 candidates are the M_0 nearest centroids and the
    search is the one-level search."""
    ps, Q, l1, l2 = _three_levels()
    ls = twolevel.LevelStack(ps, [l1, l2])
    assert [lv.nlist for lv in ls.levels] == [64, 12, 3]
    tab = aps.CapTable(ps.X.shape[1])
    p = twolevel.TwoLevelParams(k=10, recall_target=0.9, f_M=0.2, upper_recall_target=1.0, upper_f_M=1.0)
    si, _, sm, _ = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=0.9, f_M=0.2))
    for i, q in enumerate(Q):
        r0, ups = twolevel.multi_level_search_one(ls, q, p, tab)
        assert len(ups) == 2
        assert r0.ids.tolist() == si[i].tolist() and r0.m == sm[i]
