"""Pins for the oracle's estimator variants (Sec. 5.1, Table tab:recall_overhead).

APS recomputes the partition probabilities when rho moved by more than
tau_rho and reads the cap share from the table; APS-R recomputes after every
partition from the table; APS-RP recomputes after every partition with the
cap share evaluated directly.  The direct evaluation is pinned to the 3-ball
closed form; every step's estimate is recomputed here from scratch with that
closed form (p_0 = prod (1 - v_i), p_i = (1 - p_0) v_i / sum v, reading R1),
at the radius the step says it used.
"""

import math

import numpy as np
import pytest

from oracle import aps, ivf, kmeans


def ball3_cap(t):
    """Share of a unit 3-ball beyond a plane at distance t: a cap of height
    1 - t has volume pi (1 - t)^2 (2 + t) / 3, over 4 pi / 3."""
    t = np.maximum(np.asarray(t, dtype=np.float64), 0.0)
    return np.where(t < 1.0, (1.0 - np.minimum(t, 1.0)) ** 2 * (2.0 + np.minimum(t, 1.0)) / 4.0, 0.0)


def _index(d=3, n=3000, nlist=24, seed=5):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((8, d)) * 3.0
    X = (centres[rng.integers(0, 8, n)] + rng.standard_normal((n, d))).astype(np.float32)
    C = X[rng.choice(n, nlist, replace=False)].astype(np.float64)
    assign = kmeans.assign_nearest(X, C)
    ps = ivf.PartitionedSet(X, np.arange(n, dtype=np.int64) + 1000, assign, C)
    Q = (centres[rng.integers(0, 8, 40)] + rng.standard_normal((40, d))).astype(np.float32)
    return ps, Q


def _from_scratch(res, step, k, ps):
    """The estimate after `step` computed anew from the step's radius."""
    h = np.asarray(res.h, dtype=np.float64)
    scanned = res.order[: step.m]
    rows = sum(int(ps.members[int(p)].shape[0]) for p in scanned)
    if rows < k:
        return 0.0                              # reading R3
    t = np.zeros_like(h) if math.isinf(step.rho) else h / step.rho
    v = ball3_cap(t)
    V = float(v.sum())
    p0 = float(np.prod(1.0 - v))
    if not V > 0.0:
        return 1.0
    return p0 + (1.0 - p0) * float(v[: step.m - 1].sum()) / V


def test_exact_cap_is_the_function_itself():
    ts = np.linspace(0.0, 0.999, 41)
    np.testing.assert_allclose(aps.ExactCap(3)(ts), ball3_cap(ts), atol=1e-14)
    np.testing.assert_allclose(aps.ExactCap(1)(ts), 0.5 * (1.0 - ts), atol=1e-14)
    assert aps.ExactCap(64)(np.array([1.0, 2.0])).tolist() == [0.0, 0.0]
    # negative t reads as 0, as in the table
    assert aps.ExactCap(3)(np.array([-0.3]))[0] == pytest.approx(0.5, abs=1e-15)
    assert aps.CapTable(3)(np.array([-0.3]))[0] == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("every", [True, False])
def test_every_estimate_from_scratch(every):
    ps, Q = _index()
    k = 5
    prm = aps.APSParams(k=k, recall_target=0.97, f_M=1.0, tau_rho=0.3, metric="l2", recompute_every=every)
    stale = 0
    for q in Q:
        res = aps.aps_search_one(ps, q, prm, aps.ExactCap(3))
        for j, st in enumerate(res.steps):
            if every:
                assert st.recomputed and (st.rho == st.rho_new or (math.isinf(st.rho) and math.isinf(st.rho_new)))
            elif st.rho != st.rho_new:
                stale += 1
            assert st.recall == pytest.approx(_from_scratch(res, st, k, ps), abs=1e-12)
            if j + 1 < len(res.steps):
                assert st.recall < prm.recall_target
        last = res.steps[-1]
        assert last.recall >= prm.recall_target or last.m == res.order.shape[0]
    if not every:
        # with a 30% threshold some steps keep the radius of an earlier recompute
        assert stale > 0


def test_zero_threshold_equals_recompute_every():
    """tau_rho = 0 recomputes whenever rho moved at all; an unmoved rho gives
    the same probabilities, so the decisions equal the every-step variant's."""
    ps, Q = _index(d=16, seed=9)
    tab = aps.CapTable(16)
    for q in Q:
        a = aps.aps_search_one(ps, q, aps.APSParams(k=10, recall_target=0.9, f_M=0.5, tau_rho=0.0), tab)
        b = aps.aps_search_one(ps, q, aps.APSParams(k=10, recall_target=0.9, f_M=0.5, recompute_every=True), tab)
        assert a.m == b.m and a.ids.tolist() == b.ids.tolist()
        for sa, sb in zip(a.steps, b.steps):
            assert sa.recall == pytest.approx(sb.recall, abs=1e-12)


def test_table_and_direct_estimates_agree_within_interpolation_error():
    """APS-R and APS-RP differ only by the table's interpolation error, which
    for linear interpolation on a grid of step 1/1023 is below
    max|v''| / 8 * (1/1023)^2 per cap share."""
    d = 16
    ps, Q = _index(d=d, seed=11)
    tab, ex = aps.CapTable(d), aps.ExactCap(d)
    grid = np.linspace(0.0, 1.0, 200_001)
    v = ex(grid)
    curv = np.abs(np.diff(v, 2)).max() / (grid[1] - grid[0]) ** 2
    bound = curv / 8.0 / 1023.0 ** 2
    for q in Q:
        prm = aps.APSParams(k=10, recall_target=0.999, f_M=0.5, recompute_every=True)
        a = aps.aps_search_one(ps, q, prm, tab)
        b = aps.aps_search_one(ps, q, prm, ex)
        n = min(len(a.steps), len(b.steps))
        M = a.order.shape[0]
        for sa, sb in zip(a.steps[:n], b.steps[:n]):
            # p_0, and each p_i through V, move by at most M * bound each
            assert abs(sa.recall - sb.recall) <= 4.0 * M * bound + 1e-12
