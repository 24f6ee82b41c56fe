"""Pins of the maintenance oracle (Sec. 4): the cost model, the split and
delete deltas, the decision workflow and the actions on vectors.

* The paper's worked example (Sec. 4.2 "Example Maintenance Workflow"):
  the estimate is 60 - 120 + 55 = -5 us for both partitions, so both are
  split tentatively; the verify step gives -5 for the balanced 250/250
  split (commit) and +5 for the 450/50 split (reject, its children cost
  0.05 x (1050 + 250) = 65 us).
* The exact deltas equal the difference of the total cost (Eq. CostTotal,
  centroid scan included) before and after the action, summed independently
  (Eq. DeltaC).
* With a linear latency the split estimate has a closed form.
* 2-means recovers two well-separated groups; the nearest-centroid steps
  agree with brute force.
"""

import itertools

import numpy as np
import pytest

from oracle import maintenance as om


def example_latency():
    return om.Latency([50, 250, 450, 500], [250.0, 550.0, 1050.0, 1200.0])


def test_latency_table_interpolates():
    lam = example_latency()
    for s, v in [(50, 250.0), (250, 550.0), (450, 1050.0), (500, 1200.0)]:
        assert lam(s) == v
    assert lam(350) == pytest.approx(800.0, abs=1e-12)
    assert lam(25) == pytest.approx(250.0 - 25 * 300.0 / 200.0, abs=1e-12)
    with pytest.raises(ValueError):
        om.Latency([1, 1], [2, 3])


def test_worked_example_estimate():
    lam = example_latency()
    assert om.partition_cost(0.10, 500, lam) == pytest.approx(120.0, abs=1e-12)
    # each child of the balanced estimate: alpha * A = 0.05 of the queries, 250 vectors
    assert 0.05 * (lam(250) + lam(250)) == pytest.approx(55.0, abs=1e-12)
    est = om.delta_split_estimate(60.0, 0.10, 500, 0.5, lam)
    assert est == pytest.approx(-5.0, abs=1e-12)
    assert est < -4.0


def test_worked_example_verify_and_decide():
    lam = example_latency()
    outcomes = {0: om.SplitOutcome(250, 250), 1: om.SplitOutcome(450, 50)}
    dec = om.run_workflow([0.10, 0.10], [500, 500], lam, tau=4.0, alpha=0.5, dO_plus=60.0,
                          split_outcome=lambda j: outcomes[j])
    assert [(d.partition, d.action) for d in dec] == [(0, "split"), (1, "split")]
    assert dec[0].estimate == pytest.approx(-5.0, abs=1e-12)
    assert dec[1].estimate == pytest.approx(-5.0, abs=1e-12)
    assert dec[0].verified == pytest.approx(-5.0, abs=1e-12) and dec[0].committed
    assert dec[1].verified == pytest.approx(5.0, abs=1e-12) and not dec[1].committed
    # the rejected split's children: 0.05 x (1050 + 250)
    assert 0.05 * lam(450) + 0.05 * lam(50) == pytest.approx(65.0, abs=1e-12)


def test_threshold_is_strict():
    lam = example_latency()
    dec = om.run_workflow([0.10], [500], lam, tau=5.0, alpha=0.5, dO_plus=60.0,
                          split_outcome=lambda j: om.SplitOutcome(250, 250))
    assert dec == []  # -5 is not below -5


def _random_latency(rng):
    sizes = np.sort(rng.choice(np.arange(1, 5000), 6, replace=False)).astype(float)
    vals = np.cumsum(rng.uniform(1, 100, 6))
    return om.Latency(sizes, vals)


@pytest.mark.parametrize("seed", range(5))
def test_split_delta_is_the_total_cost_difference(seed):
    rng = np.random.default_rng(seed)
    lam = _random_latency(rng)
    N = 7
    A = rng.uniform(0, 1, N)
    s = rng.integers(2, 4000, N).astype(float)
    j = 3
    sL = float(rng.integers(1, s[j]))
    sR = s[j] - sL
    AL, AR = rng.uniform(0, A[j], 2)
    before = om.total_cost(A, s, lam, n_centroids=N)
    A2 = np.concatenate([np.delete(A, j), [AL, AR]])
    s2 = np.concatenate([np.delete(s, j), [sL, sR]])
    after = om.total_cost(A2, s2, lam, n_centroids=N + 1)
    dO = om.centroid_overhead_plus(N, lam)
    got = om.delta_split_exact(dO, A[j], s[j], AL, sL, AR, sR, lam)
    assert got == pytest.approx(after - before, rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("seed", range(5))
def test_merge_delta_is_the_total_cost_difference(seed):
    rng = np.random.default_rng(100 + seed)
    lam = _random_latency(rng)
    N = 8
    A = rng.uniform(0, 1, N)
    s = rng.integers(1, 3000, N).astype(float)
    j = 5
    recv = [1, 2, 6]
    share = rng.dirichlet(np.ones(len(recv)))
    ds = np.round(share * s[j])
    ds[-1] = s[j] - ds[:-1].sum()
    dA = A[j] * share
    before = om.total_cost(A, s, lam, n_centroids=N)
    A2, s2 = A.copy(), s.copy()
    for m, a, x in zip(recv, dA, ds):
        A2[m] += a
        s2[m] += x
    after = om.total_cost(np.delete(A2, j), np.delete(s2, j), lam, n_centroids=N - 1)
    dO = om.centroid_overhead_minus(N, lam)
    got = om.delta_merge_exact(dO, A[j], s[j], [(A[m], s[m], a, x) for m, a, x in zip(recv, dA, ds)], lam)
    assert got == pytest.approx(after - before, rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("alpha", [0.5, 0.9, 1.0])
def test_split_estimate_closed_form_for_linear_latency(alpha):
    a, b = 40.0, 0.75
    lam = om.Latency([0, 10_000], [a, a + b * 10_000])
    for A, s, dO in [(0.1, 500, 60.0), (0.8, 3000, 5.0), (0.02, 64, 0.3)]:
        want = dO + A * (a * (2 * alpha - 1) + b * s * (alpha - 1))
        assert om.delta_split_estimate(dO, A, s, alpha, lam) == pytest.approx(want, rel=1e-12)


def test_merge_estimate_spreads_uniformly():
    lam = example_latency()
    rec = [(0.2, 250.0), (0.1, 450.0)]
    got = om.delta_merge_estimate(-30.0, 0.05, 100.0, rec, lam)
    want = -30.0 - 0.05 * lam(100.0)
    want += (0.2 + 0.025) * lam(300.0) - 0.2 * lam(250.0)
    want += (0.1 + 0.025) * lam(500.0) - 0.1 * lam(450.0)
    assert got == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_two_means_separates_two_groups(metric):
    rng = np.random.default_rng(7)
    d = 16
    u = np.zeros(d)
    u[0] = 1.0
    v = np.zeros(d)
    v[1] = 1.0
    G0 = u + 0.05 * rng.standard_normal((40, d))
    G1 = v + 0.05 * rng.standard_normal((25, d))
    X = np.vstack([G0, G1])
    perm = rng.permutation(X.shape[0])
    X = X[perm]
    truth = (perm >= 40).astype(int)
    lab, C = om.two_means(X, X.mean(0), 8, metric)
    assert (lab == truth).all() or (lab == 1 - truth).all()
    # the left child is the group of the row farthest from the centroid
    far = np.argmax(((X - X.mean(0)) ** 2).sum(1)) if metric == "l2" else np.argmin(X @ X.mean(0))
    assert lab[far] == 0
    assert np.allclose(C[0], om._mean(X[lab == 0], metric)) and np.allclose(C[1], om._mean(X[lab == 1], metric))
    if metric == "ip":
        assert np.allclose(np.linalg.norm(C, axis=1), 1.0)


def test_two_means_is_the_best_bipartition_on_a_line():
    # tiny 1-D case: the 2-means result minimises the within-group squared
    # error over every split into two non-empty groups
    x = np.array([0.0, 0.3, 0.4, 1.1, 5.0, 5.2, 6.1, 6.3])[:, None]
    lab, _ = om.two_means(x, x.mean(0), 10, "l2")

    def sse(mask):
        return sum(((x[m] - x[m].mean(0)) ** 2).sum() for m in (mask, ~mask) if m.any())

    best = min(sse(np.array(bits, bool)) for bits in itertools.product([0, 1], repeat=len(x))
               if 0 < sum(bits) < len(x))
    assert sse(lab == 1) == pytest.approx(best, rel=1e-12)


def test_nearest_among_matches_brute_force():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, 6))
    C = rng.standard_normal((9, 6))
    allowed = [7, 1, 4, 8]
    for metric in ("l2", "ip"):
        got = om.nearest_among(X, C, allowed, metric)
        for i in range(X.shape[0]):
            if metric == "l2":
                key = [((X[i] - C[a]) ** 2).sum() for a in sorted(allowed)]
                want = sorted(allowed)[int(np.argmin(key))]
            else:
                key = [X[i] @ C[a] for a in sorted(allowed)]
                want = sorted(allowed)[int(np.argmax(key))]
            assert got[i] == want


def _blob_index(rng, n_parts, d, per_blob, hot):
    """n_parts partitions, each holding two separated blobs; `hot` partitions
    are scanned by every query of the window, the others by few."""
    centers = rng.standard_normal((2 * n_parts, d)) * 10.0
    X = np.vstack([c + rng.standard_normal((per_blob, d)) * 0.1 for c in centers])
    part = np.repeat(np.arange(n_parts), 2 * per_blob)
    C = np.stack([X[part == j].mean(0) for j in range(n_parts)])
    hits = np.where(np.isin(np.arange(n_parts), hot), 1000, 5)
    return X, part, C, hits


def test_maintain_splits_hot_partitions_and_keeps_every_row():
    rng = np.random.default_rng(11)
    X, part, C, hits = _blob_index(rng, 6, 8, 200, hot=[1, 4])
    lam = om.Latency([1, 100, 1000], [2.0, 30.0, 400.0])
    prm = om.MaintainParams(tau=1.0, alpha=0.9, refine_radius=2, refine_iters=1)
    part2, C2, dec = om.maintain(X, part, C, hits, 1000, lam, prm, "l2")
    splits = [d for d in dec if d.action == "split"]
    assert [d.partition for d in splits if d.committed] == [1, 4]
    assert C2.shape[0] == 8
    sizes = np.bincount(part2, minlength=8)
    assert sizes.sum() == X.shape[0]
    # the hot partitions' blobs now sit in partitions of their own
    for j in (1, 4):
        rows = np.nonzero(part == j)[0]
        assert len(np.unique(part2[rows[:200]])) == 1 and len(np.unique(part2[rows[200:]])) == 1
        assert part2[rows[0]] != part2[rows[-1]]
    # the cost model agrees the pass helped
    A = hits / 1000.0
    before = om.total_cost(A, np.bincount(part, minlength=6), lam, n_centroids=6)
    A2 = list(A) + [0.9 * A[1], 0.9 * A[4]]
    A2[1] *= 0.9
    A2[4] *= 0.9
    after = om.total_cost(A2, sizes, lam, n_centroids=8)
    assert after < before


def test_maintain_deletes_a_cold_tiny_partition():
    rng = np.random.default_rng(12)
    d = 8
    centers = rng.standard_normal((4, d)) * 10.0
    X = np.vstack([c + rng.standard_normal((300, d)) * 0.1 for c in centers])
    part = np.repeat(np.arange(4), 300)
    extra = centers[2] + rng.standard_normal((3, d)) * 0.1   # a stray, tiny partition near blob 2
    X = np.vstack([X, extra])
    part = np.concatenate([part, [4, 4, 4]])
    C = np.stack([X[part == j].mean(0) for j in range(5)])
    hits = np.array([100, 100, 100, 100, 0])
    # steep at small counts: one centroid fewer saves about 5.6 us
    lam = om.Latency([1, 10, 100, 1000], [0.0, 50.0, 60.0, 200.0])
    prm = om.MaintainParams(tau=0.5, alpha=0.9, refine_radius=3, merge_below=10, min_split_size=10_000)
    part2, C2, dec = om.maintain(X, part, C, hits, 100, lam, prm, "l2")
    assert [(d.partition, d.action, d.committed) for d in dec] == [(4, "merge", True)]
    assert C2.shape[0] == 4
    assert (part2[-3:] == 2).all()
    assert (part2[:-3] == part[:-3]).all()
