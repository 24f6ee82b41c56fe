"""Pins for the insert/delete replay and for the seeded generator."""

import numpy as np
import pytest

import synth
from oracle import aps, ivf, kmeans, knn, updates


def _index(n=3000, d=8, nlist=24, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    C = X[rng.choice(n, nlist, replace=False)].copy()
    a = kmeans.assign_nearest(X, C)
    r = updates.ReplayIndex(C, "l2")
    r.load(X, np.arange(n), a)
    return r, X, rng


def _search(r, Q):
    ps = r.partitioned()
    return aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=0.9, f_M=0.3))[0]


def test_insert_then_delete_restores_results():
    r, X, rng = _index()
    Q = rng.standard_normal((20, 8)).astype(np.float32)
    before = _search(r, Q)
    B = rng.standard_normal((500, 8)).astype(np.float32)
    ids = np.arange(10_000, 10_500)
    assert r.insert(B, ids) == updates.OK
    assert not (_search(r, Q) == before).all()
    assert r.delete(ids) == updates.OK
    assert (_search(r, Q) == before).all()


def test_routing_is_nearest_centroid():
    r, X, rng = _index()
    B = rng.standard_normal((200, 8)).astype(np.float32)
    r.insert(B, np.arange(50_000, 50_200))
    ps = r.partitioned()
    assert ivf.assignment_violations(ps.X, ps.assign, ps.C, "l2").size == 0


def test_state_equals_fresh_build():
    r, X, rng = _index()
    B = rng.standard_normal((300, 8)).astype(np.float32)
    r.insert(B, np.arange(7000, 7300))
    dels = rng.choice(3000, 400, replace=False)
    r.delete(dels)
    ps = r.partitioned()
    keep = np.setdiff1d(np.arange(3000), dels)
    allX = np.concatenate([X[keep], B])
    allI = np.concatenate([keep, np.arange(7000, 7300)])
    fresh = ivf.PartitionedSet(allX, allI, kmeans.assign_nearest(allX, r.C), r.C)
    Q = rng.standard_normal((10, 8)).astype(np.float32)
    a = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=0.9, f_M=0.3))[0]
    b = aps.aps_search(fresh, Q, aps.APSParams(k=10, recall_target=0.9, f_M=0.3))[0]
    assert (a == b).all()


def test_batch_rejections():
    r, X, rng = _index()
    n0 = len(r.vec)
    assert r.delete(np.array([1, 2, 999_999])) == updates.NOTFOUND
    assert r.delete(np.array([5, 5])) == updates.NOTFOUND
    assert len(r.vec) == n0
    assert r.insert(np.zeros((2, 8), np.float32), np.array([3, 77_777])) == updates.DUPLICATE
    assert r.insert(np.zeros((2, 8), np.float32), np.array([77_777, 77_777])) == updates.DUPLICATE
    assert len(r.vec) == n0


def test_delete_everything_gives_empty_results():
    r, X, rng = _index(n=500)
    assert r.delete(np.arange(500)) == updates.OK
    ps = r.partitioned()
    Q = rng.standard_normal((3, 8)).astype(np.float32)
    gi, gv, _ = ivf.ivf_search(ps, Q, 5, 24, "l2")
    assert (gi == -1).all() and np.isinf(gv).all()


def test_two_level_routing_is_top_down():
    C = np.array([[0.0, 0.0], [1.0, 0.0], [10.0, 0.0], [11.0, 0.0]], dtype=np.float32)
    C1 = np.array([[0.0, 0.0], [10.5, 0.0]], dtype=np.float32)
    r = updates.ReplayIndex(C, "l2", top_centroids=C1, top_assign=np.array([0, 0, 1, 1]))
    # (5.4, 0): the top centroid at 10.5 is nearer (5.1 vs 5.4), so the leaf is
    # chosen among {2, 3} and is 2 (4.6 away), although leaf 1 (4.4 away) is
    # the nearest leaf overall
    assert r.route(np.array([[5.4, 0.0]], np.float32)).tolist() == [2]
    assert r.route(np.array([[4.0, 0.0]], np.float32)).tolist() == [1]


def test_generator_is_deterministic_and_chunked():
    spec = synth.MixtureSpec(key=99, n=10_000, d=16, n_components=12, zipf_s=1.1, chunk=4096)
    a = synth.database(spec)
    b = synth.database(spec)
    assert (a == b).all() and a.dtype == np.float32
    _, c1 = synth.database_chunk(spec, 1)
    assert (c1 == a[4096:8192]).all()
    q1 = synth.queries(spec, 50)
    q2 = synth.queries(spec, 50)
    assert (q1 == q2).all()
    w = synth.component_weights(spec)
    assert abs(w.sum() - 1) < 1e-12 and (np.diff(w) < 0).all()


def test_generator_unit_norm_and_query_noise():
    spec = synth.MixtureSpec(key=98, n=5000, d=32, n_components=10, unit_norm=True)
    X = synth.database(spec)
    np.testing.assert_allclose(np.linalg.norm(X, axis=1), 1.0, rtol=1e-5)
    Q = synth.queries(spec, 100)
    np.testing.assert_allclose(np.linalg.norm(Q, axis=1), 1.0, rtol=1e-5)
    # each query's nearest database row is close (it was drawn around one)
    gi, gv = knn.knn_exact(X, np.arange(5000), Q, 1, "ip")
    assert (gv[:, 0] > 0.9).mean() > 0.9


def test_leaf_generator_sizes():
    ls = synth.mixture.LeafSpec(synth.MixtureSpec(key=97, n=20_000, d=8, n_components=5), n_leaves=100)
    centres, leaf_of, X = synth.leaf_spec_database(ls)
    sizes = np.bincount(leaf_of, minlength=100)
    assert sizes.sum() == 20_000 and sizes.min() >= 16 and sizes.max() > 10 * np.median(sizes)
