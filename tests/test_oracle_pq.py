"""Pins for product quantization in the oracle (Sec. 8, "Vector Compression";
readings P1-P4).

The codes are pinned by brute force (every codeword tried, ties to the
lower index) and by a lossless codebook that decodes every row exactly; the
asymmetric value (the exact value of the decoded row) by the per-subspace
table sums of the product-quantization paper, which share nothing with it;
training by Lloyd's monotone distortion and by the case where the codebook
is the rows themselves; the search by its reduction to the plain adaptive
search when the codes are lossless, and by brute force over the rows of the
partitions it scanned.
"""

import numpy as np
import pytest

from oracle import aps, ivf, kmeans, knn, pq


def lossless(rng, n, m, ds, distinct=200, lo=-4, hi=4):
    """Rows whose subvectors in each subspace are drawn from `distinct`
    small-integer vectors, and a codebook holding exactly those vectors
    (the other codewords far away)."""
    books = np.empty((m, 256, ds))
    X = np.empty((n, m * ds))
    for s in range(m):
        vals = set()
        while len(vals) < distinct:
            vals.add(tuple(rng.integers(lo, hi + 1, ds).tolist()))
        vals = np.array(sorted(vals), dtype=np.float64)
        books[s, :distinct] = vals
        books[s, distinct:] = 1000.0 + np.arange(256 - distinct)[:, None]
        X[:, s * ds:(s + 1) * ds] = vals[rng.integers(0, distinct, n)]
    return X.astype(np.float32), books


def test_encode_is_the_nearest_codeword_by_brute_force():
    rng = np.random.default_rng(1)
    m, ds = 3, 2
    books = rng.standard_normal((m, 256, ds))
    books[1, 9] = books[1, 5]            # a duplicated codeword: the lower index wins
    X = rng.standard_normal((40, m * ds))
    X[7, ds:2 * ds] = books[1, 5]
    codes = pq.encode(X, books)
    for r in range(X.shape[0]):
        for s in range(m):
            best, arg = None, -1
            for j in range(256):
                dist = sum((float(X[r, s * ds + t]) - float(books[s, j, t])) ** 2 for t in range(ds))
                if best is None or dist < best:
                    best, arg = dist, j
            assert codes[r, s] == arg
    assert codes[7, 1] == 5


def test_lossless_codebook_decodes_every_row():
    rng = np.random.default_rng(2)
    R, books = lossless(rng, 500, 4, 3)
    base = rng.integers(-20, 21, (500, 12)).astype(np.float64)   # integer centroids of the rows
    X = R + base
    codes = pq.encode(X, books, base)
    np.testing.assert_array_equal(codes, pq.encode(R, books))
    np.testing.assert_array_equal(pq.decode(codes, books, base), X)
    q = rng.integers(-4, 5, 12).astype(np.float32)
    for metric in ("l2", "ip"):
        np.testing.assert_array_equal(pq.asymmetric(q, codes, books, metric, base),
                                      knn.distances(q[None], X, metric)[0])


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_asymmetric_value_is_the_sum_of_table_entries(metric):
    """With one centroid c for the rows, the value of q and c + decoded
    residual is, per subspace, a table entry of q - c (L2), or <q, c> plus
    table entries of q (IP)."""
    rng = np.random.default_rng(3)
    m, ds = 4, 4
    books = rng.standard_normal((m, 256, ds))
    codes = rng.integers(0, 256, (300, m)).astype(np.uint8)
    q = rng.standard_normal(m * ds)
    c = rng.standard_normal(m * ds)
    got = pq.asymmetric(q, codes, books, metric, np.tile(c, (300, 1)))
    if metric == "l2":
        T = pq.tables(q - c, books, "l2")
        want = np.array([sum(T[t, codes[r, t]] for t in range(m)) for r in range(300)])
    else:
        T = pq.tables(q, books, "ip")
        want = np.array([float(q @ c) + sum(T[t, codes[r, t]] for t in range(m)) for r in range(300)])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # the subspaces are not interchangeable: reversing them changes the values
    assert not np.allclose(pq.asymmetric(q, codes[:, ::-1], books, metric, np.tile(c, (300, 1))), want)


def test_training_lowers_the_distortion():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((1500, 8)) + 3.0 * rng.integers(0, 3, (1500, 1))
    books, hist = pq.train(X, 2, 6, seed=5)
    for h in hist:
        assert (np.diff(h) <= 1e-12).all()
        assert h[-1] < h[0]
    # the last entry is the distortion of the returned codebook
    codes = pq.encode(X, books)
    err = ((X - pq.decode(codes, books)) ** 2)
    for s, h in enumerate(hist):
        assert err[:, 4 * s:4 * (s + 1)].sum(1).mean() == pytest.approx(h[-1], rel=1e-12)


def test_training_on_256_distinct_rows_keeps_them():
    rng = np.random.default_rng(6)
    X = rng.permutation(np.arange(256 * 4, dtype=np.float64)).reshape(256, 4)
    books, hist = pq.train(X, 2, 3, seed=1)
    codes = pq.encode(X, books)
    np.testing.assert_array_equal(pq.decode(codes, books), X)
    for h in hist:
        assert h[-1] == 0.0


def _index(X, nlist, seed):
    rng = np.random.default_rng(seed)
    C = X[rng.choice(X.shape[0], nlist, replace=False)].astype(np.float64)
    return ivf.PartitionedSet(X, np.arange(X.shape[0], dtype=np.int64) + 7, kmeans.assign_nearest(X, C), C)


def test_lossless_codes_give_the_plain_adaptive_search():
    """Integer centroids and residuals from a lossless codebook: every score
    is the exact distance.  (L2: the inner-product radius assumes unit-norm
    rows, which integer rows are not.)"""
    metric = "l2"
    rng = np.random.default_rng(7)
    R, books = lossless(rng, 3000, 4, 4, lo=-2, hi=2)
    C = rng.integers(-12, 13, (30, 16)).astype(np.float64)
    assign = rng.integers(0, 30, 3000)
    X = (R + C[assign]).astype(np.float32)
    ps = ivf.PartitionedSet(X, np.arange(3000, dtype=np.int64) + 7, assign, C)
    codes = pq.encode(ps.X, books, ps.C[ps.assign])
    np.testing.assert_array_equal(pq.decode(codes, books, ps.C[ps.assign]), X)
    Q = rng.integers(-12, 13, (25, 16)).astype(np.float32)
    tab = aps.CapTable(16)
    prm = aps.APSParams(k=10, recall_target=0.9, f_M=0.5, metric=metric)
    for q in Q:
        plain = aps.aps_search_one(ps, q, prm, tab)
        for keep in (10, 40):
            ri, rv, res = pq.pq_search_one(ps, codes, books, q, prm, tab, keep)
            assert res.m == plain.m
            assert ri.tolist() == plain.ids.tolist()
            np.testing.assert_array_equal(rv, plain.vals)
            for a, b in zip(res.steps, plain.steps):
                assert a.recall == b.recall


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_wide_scan_is_the_exact_rerank_of_the_best_scores(metric):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2000, 8))
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)   # the radius assumes unit-norm rows
    X = X.astype(np.float32)
    ps = _index(X, 16, 10)
    books, _ = pq.train(pq.residuals(ps), 4, 2, seed=3)
    codes = pq.encode(ps.X, books, ps.C[ps.assign])
    tab = aps.CapTable(8)
    prm = aps.APSParams(k=5, recall_target=1.0, f_M=1.0, metric=metric)
    for q in rng.standard_normal((15, 8)).astype(np.float32):
        ri, rv, res = pq.pq_search_one(ps, codes, books, q, prm, tab, 20)
        # (the estimate may reach 1 before the last candidates: their caps are empty)
        rows = np.nonzero(np.isin(ps.assign, res.order[:res.m]))[0]
        # brute force: the 20 best scores of those rows, then the 5 best exact values among them
        s = pq.asymmetric(q, codes[rows], books, metric, ps.C[ps.assign[rows]])
        key = -s if metric == "ip" else s
        cand = rows[np.lexsort((ps.ids[rows], key))[:20]]
        ex = knn.distances(q[None], ps.X[cand], metric)[0]
        ekey = -ex if metric == "ip" else ex
        best = cand[np.lexsort((ps.ids[cand], ekey))[:5]]
        assert ri.tolist() == ps.ids[best].tolist()
        # rho came from the 5th score, not from an exact value
        kth = np.sort(key)[4]
        assert res.steps[-1].rho_new == pytest.approx(aps.euclid_radius(float(-kth if metric == "ip" else kth),
                                                                        float(q.astype(np.float64) @ q), metric))


def test_fixed_nprobe_by_brute_force():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((1500, 8)).astype(np.float32)
    ps = _index(X, 12, 12)
    books, _ = pq.train(pq.residuals(ps), 2, 2, seed=4)
    codes = pq.encode(ps.X, books, ps.C[ps.assign])
    for q in rng.standard_normal((10, 8)).astype(np.float32):
        ri, rv, ci = pq.pq_nprobe_one(ps, codes, books, q, 5, 3, "l2", 15)
        d0 = ((ps.C - q.astype(np.float64)) ** 2).sum(1)
        parts = np.argsort(d0, kind="stable")[:3]
        rows = np.nonzero(np.isin(ps.assign, parts))[0]
        s = np.array([sum(float(((ps.C[ps.assign[r], 4 * t:4 * t + 4] + books[t, codes[r, t]]
                                  - q[4 * t:4 * t + 4]) ** 2).sum()) for t in range(2)) for r in rows])
        cand = rows[np.lexsort((ps.ids[rows], s))[:15]]
        assert sorted(ci.tolist()) == sorted(ps.ids[cand].tolist())
        ex = ((ps.X[cand].astype(np.float64) - q) ** 2).sum(1)
        assert ri.tolist() == ps.ids[cand][np.lexsort((ps.ids[cand], ex))[:5]].tolist()
