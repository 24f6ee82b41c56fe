"""Pins for filtered search in the oracle (Sec. 8, "Filters"; readings F1, F2).

The pass fractions are checked by counting; the scaled cap share by Monte
Carlo on its meaning (the share of passing points of a ball that lie beyond
a plane when the two sides pass at different rates); the search by exact
filtered k-NN, by the reduction to the unfiltered search when every row
passes, and by the two limits the scaling fixes (a candidate with no passing
rows is never needed; a first partition with none holds no neighbour).
"""

import math

import numpy as np
import pytest

from oracle import aps, ivf, kmeans, knn


def _index(d=8, n=4000, nlist=32, seed=3):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((10, d)) * 3.0
    X = (centres[rng.integers(0, 10, n)] + rng.standard_normal((n, d))).astype(np.float32)
    C = X[rng.choice(n, nlist, replace=False)].astype(np.float64)
    assign = kmeans.assign_nearest(X, C)
    ps = ivf.PartitionedSet(X, np.arange(n, dtype=np.int64), assign, C)
    Q = (centres[rng.integers(0, 10, 30)] + rng.standard_normal((30, d))).astype(np.float32)
    return ps, Q, rng


def test_pass_fractions_by_counting():
    ps, Q, rng = _index()
    one_hot = (np.uint32(1) << rng.integers(0, 6, ps.X.shape[0]).astype(np.uint32)).astype(np.uint32)
    for mask in (0b1, 0b101, 0b111111, 0):
        f = aps.pass_fractions(ps, one_hot, mask)
        for p in range(ps.nlist):
            rows = ps.members[p]
            exact = ((one_hot[rows] & mask) != 0).mean() if rows.size else 0.0
            assert f[p] == pytest.approx(exact, abs=1e-15)
    multi = rng.integers(0, 64, ps.X.shape[0]).astype(np.uint32)
    f = aps.pass_fractions(ps, multi, 0b110)
    for p in range(ps.nlist):
        rows = ps.members[p]
        exact = ((multi[rows] & 0b110) != 0).mean()
        assert exact - 1e-15 <= f[p] <= 1.0      # the per-bit sum bounds the union from above


@pytest.mark.parametrize("t,f1,f0", [(0.2, 0.3, 0.8), (0.5, 0.9, 0.1), (0.0, 0.5, 0.5), (0.7, 1.0, 0.2)])
def test_scaled_share_is_the_passing_share_beyond_the_plane(t, f1, f0):
    """Points uniform in a unit 3-ball; those beyond x = t pass with
    probability f1, the others with f0: the share of passing points beyond
    the plane is u = v f1 / (v f1 + (1 - v) f0)."""
    rng = np.random.default_rng(int(t * 100) + 7)
    n = 400_000
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    pts = g * (rng.random(n) ** (1.0 / 3.0))[:, None]
    beyond = pts[:, 0] > t
    passing = rng.random(n) < np.where(beyond, f1, f0)
    share = (beyond & passing).sum() / passing.sum()
    v = aps.cap_fraction(np.array([t]), 3)
    u = float(aps.filtered_share(v, np.array([f1]), f0)[0])
    sigma = math.sqrt(u * (1 - u) / passing.sum())
    assert abs(share - u) < 5 * sigma + 1e-12


def test_filtered_full_scan_is_exact_filtered_knn():
    ps, Q, rng = _index()
    attr = (np.uint32(1) << rng.integers(0, 4, ps.X.shape[0]).astype(np.uint32)).astype(np.uint32)
    tab = aps.CapTable(ps.X.shape[1])
    for i, q in enumerate(Q):
        mask = 1 << (i % 4)
        res = aps.aps_search_one(ps, q, aps.APSParams(k=10, recall_target=1.0, f_M=1.0), tab, attr=attr, mask=mask)
        keep = np.nonzero((attr & mask) != 0)[0]
        ei, ev = knn.knn_exact(ps.X[keep], keep.astype(np.int64), q[None], 10, "l2")
        assert res.ids.tolist() == ei[0].tolist()
        assert (attr[res.ids] & mask).all()


def test_everything_passing_equals_the_unfiltered_search():
    ps, Q, rng = _index(seed=8)
    attr = rng.integers(1, 2 ** 32, ps.X.shape[0], dtype=np.uint64).astype(np.uint32)
    attr[attr == 0] = 1
    tab = aps.CapTable(ps.X.shape[1])
    prm = aps.APSParams(k=10, recall_target=0.9, f_M=0.5)
    for q in Q:
        a = aps.aps_search_one(ps, q, prm, tab)
        b = aps.aps_search_one(ps, q, prm, tab, attr=attr, mask=0xFFFFFFFF)
        assert a.m == b.m and a.ids.tolist() == b.ids.tolist()
        for sa, sb in zip(a.steps, b.steps):
            assert sa.recall == pytest.approx(sb.recall, abs=1e-12)


def _two_partitions():
    # P0 around the origin, P1 around (2, 0); the query sits near the bisector x = 1
    rng = np.random.default_rng(1)
    A = rng.standard_normal((200, 2)) * 0.4
    B = rng.standard_normal((200, 2)) * 0.4 + np.array([2.0, 0.0])
    X = np.concatenate([A, B]).astype(np.float32)
    C = np.array([[0.0, 0.0], [2.0, 0.0]])
    assign = kmeans.assign_nearest(X, C)
    ps = ivf.PartitionedSet(X, np.arange(400, dtype=np.int64), assign, C)
    return ps, np.array([0.8, 0.0], dtype=np.float32)


def test_candidate_without_passing_rows_is_never_needed():
    ps, q = _two_partitions()
    attr = np.where(ps.assign == 0, 1, 2).astype(np.uint32)   # label 1 in P0, label 2 in P1
    tab = aps.CapTable(2)
    prm = aps.APSParams(k=5, recall_target=0.999, f_M=1.0)
    plain = aps.aps_search_one(ps, q, prm, tab)
    assert plain.m == 2                                         # unfiltered, P1 is needed
    res = aps.aps_search_one(ps, q, prm, tab, attr=attr, mask=1)
    assert res.m == 1 and res.steps[0].recall == pytest.approx(1.0, abs=1e-15)


def test_first_partition_without_passing_rows_holds_no_neighbour():
    ps, q = _two_partitions()
    attr = np.where(ps.assign == 0, 1, 2).astype(np.uint32)
    tab = aps.CapTable(2)
    res = aps.aps_search_one(ps, q, aps.APSParams(k=5, recall_target=0.5, f_M=1.0), tab, attr=attr, mask=2)
    # nothing passes in P0: no results, the estimate is held at 0 and P1 is scanned
    assert res.steps[0].recall == 0.0 and res.m == 2
    assert set(ps.assign[res.ids].tolist()) == {1}
    # once results exist rho is finite and P_0 carries no mass: p_0 = 0, and
    # with both candidates scanned the estimate is 1
    assert res.steps[-1].recall == pytest.approx(1.0, abs=1e-15)
