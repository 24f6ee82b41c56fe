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
    with pytest.raises(quake.QuakeError) as e:
        a.add_level(5)
    assert e.value.code == quake.E_STATE
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
