"""Batched inserts and deletes on the device against the CPU replay.

The replay starts from the device index's own centroids and placement and
applies the same batches (nearest-centroid routing, centroids fixed); after
every batch the device's stored (id, partition) pairs must equal the
replay's (routing near-ties aside) and searches must match the oracle on the
replayed state.  Also: insert-then-delete restores results bit for bit,
rejected batches change nothing, partitions that overflow move, heavy
deletes compact, and the 16-bit copy follows every change.
"""

import numpy as np
import pytest

import gpu_util as gu
import parity
from oracle import ivf as oivf
from oracle import knn as oknn
from oracle import updates as oupd

pytestmark = pytest.mark.gpu


def _state(idx):
    C, eids, epart = idx.export()
    return C.cpu().numpy(), eids.cpu().numpy(), epart.cpu().numpy()


def _replay_from(idx, metric):
    C, eids, epart = _state(idx)
    r = oupd.ReplayIndex(C, metric)
    return r, eids, epart


def _check_same_state(idx, r, metric):
    C, eids, epart = _state(idx)
    assert set(eids.tolist()) == set(r.vec.keys()), "live id sets differ"
    bad = 0
    for i, p in zip(eids.tolist(), epart.tolist()):
        if r.part[i] != p:
            # accept a near-tie in routing: both partitions equally near
            x = r.vec[i][None, :]
            d = oknn.distances(x, C[[p, r.part[i]]], metric)[0]
            scale = max(abs(d[0]), abs(d[1]), 1e-30)
            assert abs(d[0] - d[1]) <= 1e-5 * scale, f"id {i}: device partition {p}, replay {r.part[i]}"
            bad += 1
    assert bad <= 2


def _search_matches(idx, r, Q, metric, **kw):
    ps = r.partitioned()
    gi, gv, ns, _ = gu.search(idx, Q, k=10, nprobe=6, **kw)
    ri, rv, _ = oivf.ivf_search(ps, Q, 10, 6, metric)
    parity.check_all(Q, ps.X, ps.ids, gi, gv, ri, rv, metric, 10)


@pytest.fixture
def base():
    rng = np.random.default_rng(12)
    mu = rng.standard_normal((20, 24)) * 3
    X = (mu[rng.integers(0, 20, 6000)] + rng.standard_normal((6000, 24))).astype(np.float32)
    ids = rng.permutation(100_000)[:6000].astype(np.int64)
    idx = gu.build(X, ids, metric="l2", nlist=30, kmeans_iters=4, seed=1)
    r, eids, epart = _replay_from(idx, "l2")
    id_row = {int(i): k for k, i in enumerate(ids.tolist())}
    r.load(X[[id_row[i] for i in eids.tolist()]], eids, epart)
    Q = (mu[rng.integers(0, 20, 60)] + rng.standard_normal((60, 24))).astype(np.float32)
    yield idx, r, Q, rng, mu
    idx.free()


def test_insert_routes_like_the_replay(base):
    idx, r, Q, rng, mu = base
    for step in range(3):
        B = (mu[rng.integers(0, 20, 700)] + rng.standard_normal((700, 24))).astype(np.float32)
        bid = np.arange(200_000 + step * 1000, 200_000 + step * 1000 + 700, dtype=np.int64)
        idx.insert(gu.to_dev(B), gu.to_dev(bid))
        assert r.insert(B, bid) == oupd.OK
        _check_same_state(idx, r, "l2")
        _search_matches(idx, r, Q, "l2")
    assert idx.stats()[0] == len(r.vec)


def test_delete_and_compaction(base):
    idx, r, Q, rng, mu = base
    live = np.array(sorted(r.vec.keys()), dtype=np.int64)
    for frac in (0.05, 0.4, 0.3):
        live = np.array(sorted(r.vec.keys()), dtype=np.int64)
        dels = rng.choice(live, int(frac * live.size), replace=False)
        idx.delete(gu.to_dev(dels))
        assert r.delete(dels) == oupd.OK
        _check_same_state(idx, r, "l2")
        _search_matches(idx, r, Q, "l2")


def test_insert_then_delete_restores_results(base):
    idx, r, Q, rng, mu = base
    before = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.3)
    B = (mu[rng.integers(0, 20, 2000)] + rng.standard_normal((2000, 24))).astype(np.float32)
    bid = np.arange(500_000, 502_000, dtype=np.int64)
    idx.insert(gu.to_dev(B), gu.to_dev(bid))
    mid = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.3)
    assert not all((a == b).all() for a, b in zip(before, mid))
    idx.delete(gu.to_dev(bid))
    after = gu.search(idx, Q, k=10, recall_target=0.9, f_M=0.3)
    for a, b in zip(before, after):
        assert (a == b).all()


def test_rejected_batches_change_nothing(base):
    from paper_2506_03437_amd import QuakeError
    idx, r, Q, rng, mu = base
    before = gu.search(idx, Q, k=10, nprobe=5)
    n0 = idx.stats()[0]
    some = np.array(sorted(r.vec.keys())[:3], dtype=np.int64)
    x3 = np.zeros((3, 24), np.float32)
    cases = [
        ("insert", x3, np.array([900_001, 900_001, 900_002])),
        ("insert", x3, np.array([900_003, some[0], 900_004])),
        ("delete", None, np.array([some[0], 12_345_678])),
        ("delete", None, np.array([some[1], some[1]])),
    ]
    for op, x, bad in cases:
        with pytest.raises(QuakeError) as e:
            if op == "insert":
                idx.insert(gu.to_dev(x), gu.to_dev(bad.astype(np.int64)))
            else:
                idx.delete(gu.to_dev(bad.astype(np.int64)))
        assert e.value.code == (-4 if op == "insert" else -3)
    assert idx.stats()[0] == n0
    after = gu.search(idx, Q, k=10, nprobe=5)
    for a, b in zip(before, after):
        assert (a == b).all()


def test_overflowing_partition_moves(base):
    idx, r, Q, rng, mu = base
    C = r.C
    # 5,000 vectors right at one centroid: that partition must grow
    B = (C[3] + 0.01 * rng.standard_normal((5000, 24))).astype(np.float32)
    bid = np.arange(700_000, 705_000, dtype=np.int64)
    idx.insert(gu.to_dev(B), gu.to_dev(bid))
    assert r.insert(B, bid) == oupd.OK
    _check_same_state(idx, r, "l2")
    _search_matches(idx, r, np.concatenate([Q, B[:20]]), "l2")


def test_delete_everything(base):
    idx, r, Q, rng, mu = base
    allids = np.array(sorted(r.vec.keys()), dtype=np.int64)
    idx.delete(gu.to_dev(allids))
    assert idx.stats()[0] == 0
    gi, gv, ns, _ = gu.search(idx, Q, k=10, nprobe=30)
    assert (gi == -1).all() and np.isinf(gv).all()
    gi, gv, ns, _ = gu.search(idx, Q, k=10, recall_target=0.9)
    assert (gi == -1).all()


def test_updates_keep_the_16bit_copy_in_step():
    rng = np.random.default_rng(5)
    centres = rng.integers(-3, 4, (10, 32))
    X = np.clip(centres[rng.integers(0, 10, 4000)] + rng.integers(-1, 2, (4000, 32)), -4, 4).astype(np.float32)
    for metric in ("l2", "ip"):
        idx = gu.build(X, metric=metric, nlist=20, storage="bf16", kmeans_iters=3, seed=3)
        r, eids, epart = _replay_from(idx, metric)
        r.load(X[eids], eids, epart)
        B = np.clip(centres[rng.integers(0, 10, 1500)] + rng.integers(-1, 2, (1500, 32)), -4, 4).astype(np.float32)
        bid = np.arange(10_000, 11_500, dtype=np.int64)
        idx.insert(gu.to_dev(B), gu.to_dev(bid))
        r.insert(B, bid)
        dels = rng.choice(np.array(sorted(r.vec.keys())), 1800, replace=False)
        idx.delete(gu.to_dev(dels))
        r.delete(dels)
        Q = np.clip(centres[rng.integers(0, 10, 40)] + rng.integers(-1, 2, (40, 32)), -4, 4).astype(np.float32)
        _check_same_state(idx, r, metric)
        # search over the device's own placement (routing near-ties aside it is the replay's)
        C, eids, epart = _state(idx)
        ps = oivf.PartitionedSet(np.stack([r.vec[i] for i in eids.tolist()]), eids, epart, C)
        gi, gv, _, _ = gu.search(idx, Q, k=10, nprobe=6, scan_mode="batched", scan_dtype="bf16")
        ri, rv, _ = oivf.ivf_search(ps, Q, 10, 6, metric)
        parity.check_all(Q, ps.X, ps.ids, gi, gv, ri, rv, metric, 10)
        idx.free()


def test_repeated_overflow_repacks_the_arena(base):
    """Growing partitions move to fresh tiles and leave their old ones behind;
    once those make up a quarter of the arena an insert packs the partitions
    into a fresh arena instead of growing it.  The state and the searches
    still follow the replay, and device memory stays bounded."""
    idx, r, Q, rng, mu = base
    C = r.C
    # one partition keeps growing: each move leaves its previous tiles behind,
    # a third of the arena after a few batches
    for step in range(12):
        B = (C[3] + 0.01 * rng.standard_normal((1500, 24))).astype(np.float32)
        bid = np.arange(800_000 + step * 2000, 800_000 + step * 2000 + 1500, dtype=np.int64)
        idx.insert(gu.to_dev(B), gu.to_dev(bid))
        assert r.insert(B, bid) == oupd.OK
        if step % 3 == 2:
            _check_same_state(idx, r, "l2")
            _search_matches(idx, r, np.concatenate([Q, B[:10]]), "l2")
    dels = np.arange(800_000, 800_000 + 1500, dtype=np.int64)
    idx.delete(gu.to_dev(dels))
    assert r.delete(dels) == oupd.OK
    _check_same_state(idx, r, "l2")
    _search_matches(idx, r, Q, "l2")
