"""Adding and removing a level (Sec. 4.2, "Add Level", "Remove Level",
"Adding and Removing Levels").

Adding a level to a one-level index must give the index that a two-level
build over the same level 0 gives (the same level-1 centroids and top
partition of every level-0 centroid, bit for bit, and the same searches);
removing it must give back the one-level index's searches bit for bit.  The
thresholds act as stated, inserts after an added level route top-down, and
the level-1 partitioning places every level-0 centroid in its nearest top
partition.
"""

import numpy as np
import pytest

import gpu_util as gu
import synth
from oracle import ivf as oivf

pytestmark = pytest.mark.gpu

UP = dict(upper_recall_target=0.99, upper_f_M=0.25)


def _data():
    spec = synth.MixtureSpec(key=61, n=40_000, d=32, n_components=50, zipf_s=1.1)
    return synth.database(spec), synth.queries(spec, 200)


def _same(ra, rb):
    for x, y in zip(ra, rb):
        assert (x == y).all()


def test_add_then_remove_level():
    from paper_2506_03437_amd import quake
    X, Q = _data()
    print("[build] one level, 400 partitions", flush=True)
    a = gu.build(X, metric="l2", nlist=400, kmeans_iters=5, seed=3)
    flat = gu.search(a, Q, k=10, recall_target=0.9, f_M=0.05)
    C, ids, part = a.export()
    # the same level 0 built with two levels from the start (export lists
    # ids and partitions in store order; the build takes the row order)
    assign = np.empty(X.shape[0], dtype=np.int32)
    assign[ids.cpu().numpy()] = part.cpu().numpy()
    b = gu.build(X, metric="l2", nlist=400, n_levels=2, nlist_top=20, kmeans_iters=5, seed=11,
                 centroids=C, assign=gu.to_dev(assign))
    a.add_level(20, kmeans_iters=5, seed=11)
    assert a.describe()["n_levels"] == 2
    Ta, ta = quake.quake_export_top(a.handle, 32, 20)
    Tb, tb = quake.quake_export_top(b.handle, 32, 20)
    assert (Ta.cpu().numpy() == Tb.cpu().numpy()).all() and (ta.cpu().numpy() == tb.cpu().numpy()).all()
    bad = oivf.assignment_violations(C.cpu().numpy(), ta.cpu().numpy().astype(np.int64), Ta.cpu().numpy(), "l2",
                                     rtol=1e-5)
    assert bad.size == 0
    _same(gu.search(a, Q, k=10, recall_target=0.9, f_M=0.05, **UP),
          gu.search(b, Q, k=10, recall_target=0.9, f_M=0.05, **UP))
    a.add_level(5, kmeans_iters=3, seed=1)                  # a third level
    assert a.level_sizes() == [400, 20, 5]
    with pytest.raises(quake.QuakeError) as e:
        a.add_level(2)                                       # at most three
    assert e.value.code == quake.E_STATE
    a.remove_level()
    a.remove_level()
    assert a.describe()["n_levels"] == 1
    _same(gu.search(a, Q, k=10, recall_target=0.9, f_M=0.05), flat)
    with pytest.raises(quake.QuakeError) as e:
        a.remove_level()
    assert e.value.code == quake.E_STATE
    a.free()
    b.free()


def test_thresholds_and_inserts_after_adding():
    X, Q = _data()
    print("[build] thresholds", flush=True)
    a = gu.build(X, metric="l2", nlist=400, kmeans_iters=5, seed=3)
    assert a.adjust_levels(add_above=400) == 0          # 400 partitions: not above the threshold
    assert a.adjust_levels(add_above=399) == 1          # sqrt(400) = 20 top partitions
    assert a.describe()["n_levels"] == 2
    from paper_2506_03437_amd import quake
    T, top = quake.quake_export_top(a.handle, 32, 20)
    assert T.shape[0] == 20
    assert a.adjust_levels(remove_below=20) == 0        # 20 top partitions: not below
    # inserts route top-down: nearest top partition, then its nearest leaf
    rng = np.random.default_rng(1)
    Xn = (X[rng.choice(X.shape[0], 500, replace=False)] + 0.05 * rng.standard_normal((500, 32))).astype(np.float32)
    ids_n = np.arange(10 ** 6, 10 ** 6 + 500, dtype=np.int64)
    a.insert(gu.to_dev(Xn), gu.to_dev(ids_n))
    C, eids, epart = a.export()
    C, eids, epart = C.cpu().numpy().astype(np.float64), eids.cpu().numpy(), epart.cpu().numpy()
    T, top = T.cpu().numpy().astype(np.float64), top.cpu().numpy()
    leaf_of = dict(zip(eids.tolist(), epart.tolist()))
    for r in range(Xn.shape[0]):
        x = Xn[r].astype(np.float64)
        dt = ((T - x) ** 2).sum(1)
        t = int(np.argmin(dt))
        leaves = np.nonzero(top == t)[0]
        dl = ((C[leaves] - x) ** 2).sum(1)
        gap_t = np.sort(dt)[1] - dt.min() if T.shape[0] > 1 else np.inf
        gap_l = np.sort(dl)[1] - dl.min() if leaves.size > 1 else np.inf
        if min(gap_t, gap_l) <= 1e-4 * dl.min():
            continue  # a near tie in FP32: either side is right
        assert leaf_of[int(ids_n[r])] == int(leaves[np.argmin(dl)])
    assert a.adjust_levels(remove_below=21) == -1
    assert a.describe()["n_levels"] == 1
    assert a.stats()[0] == X.shape[0] + 500
    a.free()


@pytest.fixture(scope="module")
def three_levels():
    spec = synth.MixtureSpec(key=62, n=60_000, d=32, n_components=60, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 200)
    print("[build] three levels: 900 leaves, 60 and 8 upper partitions", flush=True)
    idx = gu.build(X, metric="l2", nlist=900, n_levels=2, nlist_top=60, kmeans_iters=5, seed=7)
    before = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, **UP)
    idx.add_level(8, kmeans_iters=5, seed=9)
    assert idx.describe()["n_levels"] == 3 and idx.level_sizes() == [900, 60, 8]
    from oracle import twolevel as otl
    leaves = gu.oracle_view(idx, X)
    C1, a1 = idx.export_level(1)
    C2, a2 = idx.export_level(2)
    ls = otl.LevelStack(leaves, [(a1.cpu().numpy().astype(np.int64), C1.cpu().numpy()),
                                 (a2.cpu().numpy().astype(np.int64), C2.cpu().numpy())])
    yield X, Q, idx, ls, before
    idx.free()


def test_three_level_partitionings_are_nearest(three_levels):
    X, Q, idx, ls, before = three_levels
    for lv in (1, 2):
        up = ls.levels[lv]
        bad = oivf.assignment_violations(up.X, up.assign, up.C, "l2", rtol=1e-5)
        assert bad.size == 0


def test_three_levels_with_exact_upper_levels_equal_one_level(three_levels):
    import parity
    from oracle import aps as oaps
    X, Q, idx, ls, before = three_levels
    gi, gv, ns, _ = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, upper_recall_target=1.0, upper_f_M=1.0)
    table = oaps.CapTable(X.shape[1])
    params = oaps.APSParams(k=10, recall_target=0.9, f_M=0.05, metric="l2")
    id_to_row = {i: i for i in range(X.shape[0])}
    for i in range(Q.shape[0]):
        res = oaps.aps_search_one(ls.levels[0], Q[i], params, table)
        ri, rv = oivf.scan_partitions(ls.levels[0], Q[i], res.order[: ns[i]], 10, "l2")
        parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")


def test_three_levels_follow_the_oracle(three_levels):
    """The device's level-0 candidate list is the oracle's top-down result
    (APS at each level at target 0.99 over 25% of the partitions) except for
    queries decided at a near tie or within the margin at an upper level,
    and the results are exactly the top-k over the partitions scanned."""
    import parity
    from oracle import aps as oaps
    from oracle import twolevel as otl
    X, Q, idx, ls, before = three_levels
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, **UP)
    order, h = idx.candidates(gu.to_dev(Q), 0.05, **UP)
    order = order.cpu().numpy()
    table = oaps.CapTable(X.shape[1])
    p = otl.TwoLevelParams(k=10, recall_target=0.9, f_M=0.05, upper_recall_target=0.99, upper_f_M=0.25)
    id_to_row = {i: i for i in range(X.shape[0])}
    same = 0
    for i in range(Q.shape[0]):
        dev = order[i][order[i] >= 0].astype(np.int64)
        m = int(ns[i])
        ri, rv = oivf.scan_partitions(ls.levels[0], Q[i], dev[:m], 10, "l2")
        parity.check_topk(Q[i], X, id_to_row, gi[i], gv[i], ri, rv, "l2", 10, f"query {i}")
        r0, ups = otl.multi_level_search_one(ls, Q[i], p, table)
        same += set(dev.tolist()) == set(ups[-1].ids[ups[-1].ids >= 0].tolist())
    assert same >= 0.95 * Q.shape[0], same


def test_three_level_inserts_route_top_down_and_removal(three_levels, tmp_path):
    from paper_2506_03437_amd import Index
    X, Q, idx, ls, before = three_levels
    rng = np.random.default_rng(4)
    Xn = (X[rng.choice(X.shape[0], 300, replace=False)] + 0.05 * rng.standard_normal((300, 32))).astype(np.float32)
    ids_n = np.arange(10 ** 6, 10 ** 6 + 300, dtype=np.int64)
    idx.insert(gu.to_dev(Xn), gu.to_dev(ids_n))
    C, eids, epart = idx.export()
    leaf_of = dict(zip(eids.cpu().numpy().tolist(), epart.cpu().numpy().tolist()))
    L1, L2 = ls.levels[1], ls.levels[2]
    checked = 0
    for r in range(Xn.shape[0]):
        x = Xn[r].astype(np.float64)
        path, near = [], False
        cand = np.arange(L2.nlist)
        for lv, (C_, members) in ((2, (L2.C, None)), (1, (L1.C, None)), (0, (ls.levels[0].C, None))):
            dist = ((np.asarray(C_, dtype=np.float64)[cand] - x) ** 2).sum(1)
            srt = np.sort(dist)
            if srt.size > 1 and srt[1] - srt[0] <= 1e-4 * max(srt[0], 1e-12):
                near = True
            pick = int(cand[np.argmin(dist)])
            path.append(pick)
            if lv == 2:
                cand = np.nonzero(L2.assign == pick)[0]
            elif lv == 1:
                cand = np.nonzero(L1.assign == pick)[0]
            if cand.size == 0:
                near = True
                break
        if near:
            continue
        assert leaf_of[int(ids_n[r])] == path[-1], f"row {r}"
        checked += 1
    assert checked >= 0.9 * Xn.shape[0]
    # a save and load keeps all three levels
    path = str(tmp_path / "three.qk")
    idx.save(path)
    b = Index.load(path)
    assert b.level_sizes() == [900, 60, 8]
    _same(gu.search(b, Q, k=10, recall_target=0.9, f_M=0.05, **UP),
          gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, **UP))
    b.free()
    idx.delete(gu.to_dev(ids_n))
    # removing the third level gives back the two-level searches
    idx.remove_level()
    assert idx.level_sizes() == [900, 60, 0]
    _same(gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.05, **UP), before)
