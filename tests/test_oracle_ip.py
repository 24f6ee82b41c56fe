"""Pins for the inner-product branches of the oracle.

On unit-norm vectors and unit-norm centroids the squared Euclidean distance
is |q|^2 + 1 - 2 q.x, so the inner-product reading of Adaptive Partition
Scanning (Sec. 5; the bisector of c_0 and c_i is the inner-product cell
boundary, and rho is the Euclidean radius implied by the k-th score) must
reproduce the L2 algorithm step for step: the same candidate order, the
same bisector distances, the same rho after every partition, the same
recall estimates, the same stop count and the same ids.  This ties every
inner-product formula of the oracle (scores, ordering keys, h, rho) to the
L2 branch, which the geometric pins elsewhere fix independently.

The inner-product placement check is pinned by a planted mistake: a row
put in a centroid that is not its best by inner product must be reported,
and a correct placement must not.
"""

import math

import numpy as np
import pytest

from oracle import aps, ivf, knn


def _unit(a):
    a = np.asarray(a, dtype=np.float64)
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _unit_sphere_index(seed, n=3000, d=12, comps=15, nlist=30, nq=40):
    """FP64 unit vectors in clusters, unit centroids, IP-nearest placement."""
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((comps, d))
    X = _unit(mu[rng.integers(0, comps, n)] + 0.35 * rng.standard_normal((n, d)))
    C = _unit(X[rng.choice(n, nlist, replace=False)] + 0.05 * rng.standard_normal((nlist, d)))
    assign = np.argmax(X @ C.T, axis=1)
    Q = _unit(X[rng.choice(n, nq, replace=False)] + 0.15 * rng.standard_normal((nq, d)))
    ids = rng.permutation(10 * n)[:n].astype(np.int64)
    return ivf.PartitionedSet(X, ids, assign, C), Q


def test_unit_norm_l2_and_ip_cells_coincide():
    ps, _ = _unit_sphere_index(0)
    a_l2 = np.argmin(knn.distances(ps.X, ps.C, "l2"), axis=1)
    assert (a_l2 == ps.assign).all()


@pytest.mark.parametrize("seed,tau,f_M,k", [(1, 0.8, 0.3, 10), (2, 0.9, 0.5, 5), (3, 0.95, 0.2, 20),
                                           (4, 0.99, 1.0, 10)])
def test_ip_search_replays_l2_search_on_the_unit_sphere(seed, tau, f_M, k):
    ps, Q = _unit_sphere_index(seed)
    table = aps.CapTable(ps.X.shape[1])
    pl = aps.APSParams(k=k, recall_target=tau, f_M=f_M, metric="l2")
    pi = aps.APSParams(k=k, recall_target=tau, f_M=f_M, metric="ip")
    ms = []
    for i in range(Q.shape[0]):
        rl = aps.aps_search_one(ps, Q[i], pl, table)
        ri = aps.aps_search_one(ps, Q[i], pi, table)
        assert rl.order.tolist() == ri.order.tolist(), f"query {i}: candidate order"
        np.testing.assert_allclose(ri.h, rl.h, rtol=0, atol=1e-12)
        assert ri.m == rl.m, f"query {i}: stop count {ri.m} vs {rl.m}"
        assert ri.ids.tolist() == rl.ids.tolist(), f"query {i}: ids"
        # scores and squared distances are the same numbers in another form
        np.testing.assert_allclose(2.0 - 2.0 * ri.vals, rl.vals, rtol=0, atol=1e-12)
        for a, b in zip(rl.steps, ri.steps):
            assert a.recomputed == b.recomputed
            if math.isfinite(a.rho):
                assert abs(a.rho - b.rho) < 1e-12 and abs(a.rho_new - b.rho_new) < 1e-12
            assert abs(a.recall - b.recall) < 1e-9
        ms.append(rl.m)
    # the queries exercise the recall model (not every query stops at P_0)
    assert max(ms) > 1


def test_ip_radius_is_the_euclidean_distance_of_the_kth_result():
    """For a unit-norm row x, |q - x| follows from the score alone."""
    rng = np.random.default_rng(5)
    X = _unit(rng.standard_normal((50, 9)))
    q = rng.standard_normal(9) * 1.7
    s = X @ q
    for x, v in zip(X, s):
        assert abs(aps.euclid_radius(float(v), float(q @ q), "ip") - np.linalg.norm(q - x)) < 1e-12


def test_ip_bisector_is_distance_to_the_cell_boundary():
    """h_i is the distance from q to the hyperplane where c_0 and c_i score equally."""
    rng = np.random.default_rng(6)
    C = _unit(rng.standard_normal((6, 7)))
    for _ in range(20):
        q = rng.standard_normal(7)
        vals = C @ q
        c0 = int(np.argmax(vals))
        others = np.array([j for j in range(6) if j != c0])
        h = aps.bisector_distances(q, C, vals, c0, others, "ip")
        for hi, j in zip(h, others):
            w = C[c0] - C[j]
            # project q onto the plane w.x = 0 and measure the step
            foot = q - (w @ q) / (w @ w) * w
            assert abs(foot @ C[c0] - foot @ C[j]) < 1e-12
            assert hi >= 0 and abs(hi - np.linalg.norm(q - foot)) < 1e-12


def test_ip_placement_check_reports_a_planted_mistake():
    rng = np.random.default_rng(9)
    C = _unit(rng.standard_normal((8, 10)))
    X = _unit(C[rng.integers(0, 8, 400)] + 0.2 * rng.standard_normal((400, 10)))
    good = np.argmax(X @ C.T, axis=1)
    assert ivf.assignment_violations(X, good, C, "ip").size == 0
    bad = good.copy()
    planted = [17, 230]
    for r in planted:
        bad[r] = int(np.argmin(X[r] @ C.T))   # its worst centroid by inner product
    assert ivf.assignment_violations(X, bad, C, "ip").tolist() == planted
    # a near-tie within the tolerance is accepted either way
    Ct = C.copy()
    Ct[1] = Ct[0]
    Xt = np.repeat(Ct[:1], 3, axis=0)
    assert ivf.assignment_violations(Xt, np.array([0, 1, 0]), Ct, "ip").size == 0


def test_ip_fixed_nprobe_takes_the_highest_scoring_centroids():
    ps, Q = _unit_sphere_index(7)
    ids, vals, probes = ivf.ivf_search(ps, Q, 10, 4, "ip")
    for i in range(Q.shape[0]):
        s = ps.C @ Q[i]
        want = np.lexsort((np.arange(s.shape[0]), -s))[:4]
        assert probes[i].tolist() == want.tolist()
        assert (np.diff(vals[i]) <= 0).all()


def test_calibration_band_inner_product_d768():
    """P6 on a reduced d = 768 inner-product mixture (unit-norm rows, Zipf
    components, spherical k-means into 400 partitions of about 250 rows):
    mean recall@10 stays within 0.02 below the target.  On denser
    partitionings of the same generator the cap model under-delivers at
    high targets (a property of the model on this data, measured and
    recorded with the design notes, not a pinned value)."""
    import synth
    spec = synth.MixtureSpec(key=77, n=100_000, d=768, n_components=400, zipf_s=1.1, unit_norm=True)
    X = synth.database(spec)
    Q = synth.queries(spec, 300)
    rng = np.random.default_rng(0)
    C = X[rng.choice(X.shape[0], 400, replace=False)].astype(np.float64)
    for _ in range(8):
        a = np.argmax(X @ C.T.astype(np.float32), 1)
        for j in range(C.shape[0]):
            s = a == j
            if s.any():
                C[j] = X[s].astype(np.float64).mean(0)
        C /= np.linalg.norm(C, axis=1, keepdims=True)
    a = np.argmax(X.astype(np.float64) @ C.T, 1)
    ps = ivf.PartitionedSet(X, np.arange(X.shape[0]), a, C)
    truth, _ = knn.knn_exact(X, ps.ids, Q, 10, "ip")
    table = aps.CapTable(768)
    prev = 0.0
    for tau in (0.8, 0.9, 0.95):
        gi, _, _, _ = aps.aps_search(ps, Q, aps.APSParams(k=10, recall_target=tau, f_M=0.125, metric="ip"), table)
        rec = float(knn.recall_at_k(gi, truth, 10).mean())
        assert rec >= tau - 0.02, (tau, rec)
        assert rec >= prev
        prev = rec


def test_ip_multi_level_search_replays_l2_on_the_unit_sphere():
    """The level hand-over keeps the metric: with unit vectors and unit
    centroids at every level, the three-level search in inner product takes
    the same candidates, stops and results as in L2."""
    from oracle import twolevel
    ps, Q = _unit_sphere_index(5, n=4000, nlist=60)
    rng = np.random.default_rng(6)
    C1 = _unit(ps.C[rng.choice(60, 10, replace=False)] + 0.05 * rng.standard_normal((10, ps.C.shape[1])))
    a1 = np.argmax(ps.C @ C1.T, axis=1)
    C2 = _unit(C1[rng.choice(10, 3, replace=False)] + 0.05 * rng.standard_normal((3, ps.C.shape[1])))
    a2 = np.argmax(C1 @ C2.T, axis=1)
    ls = twolevel.LevelStack(ps, [(a1, C1), (a2, C2)])
    table = aps.CapTable(ps.X.shape[1])
    pl = twolevel.TwoLevelParams(k=10, recall_target=0.9, f_M=0.2, upper_recall_target=0.99, upper_f_M=0.5,
                                 metric="l2")
    pi = twolevel.TwoLevelParams(k=10, recall_target=0.9, f_M=0.2, upper_recall_target=0.99, upper_f_M=0.5,
                                 metric="ip")
    for q in Q:
        rl, ul = twolevel.multi_level_search_one(ls, q, pl, table)
        ri, ui = twolevel.multi_level_search_one(ls, q, pi, table)
        for a, b in zip(ul, ui):
            assert a.ids.tolist() == b.ids.tolist() and a.m == b.m
        assert rl.order.tolist() == ri.order.tolist() and rl.m == ri.m
        assert rl.ids.tolist() == ri.ids.tolist()
