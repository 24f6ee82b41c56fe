"""Host-side helpers of the benchmark, checked on the CPU.

The per-query oracle nprobe of the early-termination comparison (Sec. 7,
Table tab:early_term) is checked by brute force: scanning that many nearest
partitions with the oracle's IVF search finds at least `need` of the query's
true neighbours, and one partition fewer does not.
"""

import numpy as np
import pytest

import bench
from oracle import ivf, kmeans, knn


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_min_nprobe_per_query_by_brute_force(metric):
    rng = np.random.default_rng(4)
    n, d, nlist, k = 4000, 12, 40, 10
    X = (rng.standard_normal((n, d)) + 2.0 * rng.standard_normal((8, d))[rng.integers(0, 8, n)]).astype(np.float32)
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    C = X[rng.choice(n, nlist, replace=False)].astype(np.float64)
    assign = kmeans.assign_nearest(X, C) if metric == "l2" else np.argmax(X.astype(np.float64) @ C.T, axis=1)
    ps = ivf.PartitionedSet(X, np.arange(n), assign, C)
    Q = X[rng.choice(n, 30, replace=False)] + 0.05 * rng.standard_normal((30, d)).astype(np.float32)
    truth, _ = knn.knn_exact(X, np.arange(n), Q, k, metric)
    key = knn.sort_key(knn.distances(Q, C, metric), metric)
    for need in (1, 8, 9, 10):
        got = bench.min_nprobe_per_query(key, np.asarray(assign), truth, need)
        for i in range(Q.shape[0]):
            order = np.argsort(key[i], kind="stable")
            held = lambda m: len(set(np.concatenate([ps.members[p] for p in order[:m]]).tolist())
                                 & set(truth[i].tolist()))
            assert held(got[i]) >= need
            assert got[i] == 1 or held(got[i] - 1) < need
