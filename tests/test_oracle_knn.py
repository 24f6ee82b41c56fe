"""Pins for the exact k-NN, fixed-nprobe and assignment parts of the oracle.

Each check ties the oracle to something other than itself: pure-Python
brute force on tiny inputs, the nprobe = N_l invariant, monotonicity of
recall in nprobe, tie-breaking by id, and a planted assignment mistake.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import ivf, kmeans, knn



def _py_l2(q, x):
    return sum((float(a) - float(b)) ** 2 for a, b in zip(q, x))


def _py_ip(q, x):
    return sum(float(a) * float(b) for a, b in zip(q, x))


def _py_knn(X, ids, q, k, metric):
    rows = []
    for i, x in zip(ids, X):
        v = _py_l2(q, x) if metric == "l2" else _py_ip(q, x)
        rows.append(((v if metric == "l2" else -v), int(i), v))
    rows.sort()
    return [r[1] for r in rows[:k]], [r[2] for r in rows[:k]]


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_knn_matches_pure_python(metric):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((60, 5)).astype(np.float32)
    ids = rng.permutation(1000)[:60].astype(np.int64)
    Q = rng.standard_normal((9, 5)).astype(np.float32)
    got_i, got_v = knn.knn_exact(X, ids, Q, 7, metric, row_block=17, query_block=4)
    for j in range(Q.shape[0]):
        ei, ev = _py_knn(X, ids, Q[j], 7, metric)
        assert list(got_i[j]) == ei
        np.testing.assert_allclose(got_v[j], ev, rtol=1e-12, atol=1e-12)


def test_l2_forms_agree():
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((200, 64)) + 5).astype(np.float32)
    Q = (rng.standard_normal((20, 64)) + 5).astype(np.float32)
    a = knn.l2_direct(Q, X)
    b = knn.l2_expanded(Q, X)
    np.testing.assert_allclose(a, b, rtol=1e-10)


def test_ties_go_to_lower_id():
    X = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]], dtype=np.float32)
    ids = np.array([40, 10, 30, 20])
    q = np.zeros((1, 2), dtype=np.float32)
    i, v = knn.knn_exact(X, ids, q, 3, "l2")
    assert list(i[0]) == [10, 20, 30]
    assert list(v[0]) == [1.0, 1.0, 1.0]


def test_fewer_than_k_pads():
    X = np.ones((2, 3), dtype=np.float32)
    i, v = knn.knn_exact(X, np.array([5, 6]), np.zeros((1, 3), np.float32), 4, "l2")
    assert list(i[0]) == [5, 6, -1, -1]
    assert math.isinf(v[0, 3])
    i, v = knn.knn_exact(X, np.array([5, 6]), np.zeros((1, 3), np.float32), 4, "ip")
    assert v[0, 3] == -np.inf


def test_permutation_invariance():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((300, 8)).astype(np.float32)
    ids = np.arange(300)
    Q = rng.standard_normal((5, 8)).astype(np.float32)
    a, _ = knn.knn_exact(X, ids, Q, 10, "l2")
    p = rng.permutation(300)
    b, _ = knn.knn_exact(X[p], ids[p], Q, 10, "l2")
    assert (a == b).all()


def _tiny_index(metric, n=400, d=6, nlist=12, seed=5):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    C = X[rng.choice(n, nlist, replace=False)].copy()
    a = kmeans.assign_nearest(X, C) if metric == "l2" else np.argmax(X.astype(np.float64) @ C.T.astype(np.float64), 1)
    return X, np.arange(n), a, C


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_ivf_all_partitions_equals_exact(metric):
    X, ids, a, C = _tiny_index(metric)
    Q = np.random.default_rng(1).standard_normal((15, X.shape[1])).astype(np.float32)
    ps = ivf.PartitionedSet(X, ids, a, C)
    gi, gv, _ = ivf.ivf_search(ps, Q, 10, C.shape[0], metric)
    ei, ev = knn.knn_exact(X, ids, Q, 10, metric)
    assert (gi == ei).all()
    np.testing.assert_allclose(gv, ev)


def test_ivf_matches_pure_python_probe():
    X, ids, a, C = _tiny_index("l2")
    Q = np.random.default_rng(2).standard_normal((6, X.shape[1])).astype(np.float32)
    ps = ivf.PartitionedSet(X, ids, a, C)
    gi, _, probes = ivf.ivf_search(ps, Q, 5, 3, "l2")
    for j in range(Q.shape[0]):
        cd = sorted((_py_l2(Q[j], c), p) for p, c in enumerate(C))
        probe = [p for _, p in cd[:3]]
        assert list(probes[j]) == probe
        sel = [i for i in range(X.shape[0]) if a[i] in probe]
        ei, _ = _py_knn(X[sel], ids[sel], Q[j], 5, "l2")
        assert list(gi[j]) == ei


def test_recall_non_decreasing_in_nprobe():
    X, ids, a, C = _tiny_index("l2", n=800, nlist=20)
    Q = np.random.default_rng(4).standard_normal((25, X.shape[1])).astype(np.float32)
    ps = ivf.PartitionedSet(X, ids, a, C)
    truth, _ = knn.knn_exact(X, ids, Q, 10, "l2")
    prev = np.zeros(Q.shape[0])
    for nprobe in range(1, 21):
        gi, _, _ = ivf.ivf_search(ps, Q, 10, nprobe, "l2")
        rec = knn.recall_at_k(gi, truth, 10)
        assert (rec >= prev - 1e-12).all()
        prev = rec
    assert (prev == 1.0).all()


def test_recall_definition():
    found = np.array([[1, 2, 3, -1], [4, 5, 6, 7]])
    truth = np.array([[3, 2, 9, 8], [7, 6, 5, 4]])
    np.testing.assert_allclose(knn.recall_at_k(found, truth, 4), [0.5, 1.0])


def test_assignment_check_flags_planted_mistake():
    X, ids, a, C = _tiny_index("l2")
    assert ivf.assignment_violations(X, a, C, "l2").size == 0
    bad = a.copy()
    bad[17] = (bad[17] + 1) % C.shape[0]
    v = ivf.assignment_violations(X, bad, C, "l2")
    assert list(v) == [17]


def test_lloyd_objective_non_increasing():
    rng = np.random.default_rng(9)
    X = np.concatenate([rng.standard_normal((50, 3)) + c for c in ([0, 0, 0], [6, 0, 0], [0, 6, 0])])
    _, _, hist = kmeans.lloyd(X, X[[0, 1, 2]], 8)
    for a, b in itertools.pairwise(hist) if hasattr(itertools, "pairwise") else zip(hist, hist[1:]):
        assert b <= a + 1e-9
