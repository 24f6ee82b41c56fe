"""How the work is cut (items per partition, windows, item-buffer size)
must never change a result: partitions are committed in candidate order
whatever the schedule.  Also parity on partitions much larger than one work
item, so that one partition's results arrive in several pieces."""

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import ivf as oivf
from oracle import knn as oknn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big_parts():
    spec = synth.MixtureSpec(key=31, n=150_000, d=64, n_components=40, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 400)
    print("[build] 150k x 64, 24 partitions (several work items each)", flush=True)
    idx = gu.build(X, metric="l2", nlist=24, kmeans_iters=5, seed=4)
    ps = gu.oracle_view(idx, X)
    assert ps.sizes().max() > 16 * 64 * 3
    yield X, Q, idx, ps
    idx.free()


SCHEDULES = [dict(chunk_tiles=1), dict(max_items=1), dict(first_window=1, max_window=1), dict(first_window=8),
             dict(chunk_tiles=3, max_items=50), dict(chunk_tiles=200), dict(rounds_per_sync=1, blocks_per_cu=1),
             dict(rounds_per_sync=16, blocks_per_cu=32), dict(no_graph=1, rounds_per_sync=3)]


@pytest.mark.parametrize("mode", [dict(recall_target=0.9, f_M=0.5), dict(nprobe=5), dict(recall_target=0.99, f_M=1.0)])
def test_schedule_never_changes_results(big_parts, mode):
    X, Q, idx, ps = big_parts
    idx.set_tuning()
    base = gu.search(idx, Q, k=20, **mode)
    for sch in SCHEDULES:
        idx.set_tuning(**sch)
        got = gu.search(idx, Q, k=20, **mode)
        for a, b in zip(base, got):
            assert (a == b).all(), f"schedule {sch} changed the result"
    idx.set_tuning()


def test_multi_item_partitions_match_oracle(big_parts):
    X, Q, idx, ps = big_parts
    gi, gv, ns, _ = gu.search(idx, Q, k=10, nprobe=3)
    ri, rv, _ = oivf.ivf_search(ps, Q, 10, 3, "l2")
    parity.check_all(Q, X, ps.ids, gi, gv, ri, rv, "l2", 10)
    idx.set_tuning(chunk_tiles=1, max_items=1)
    gi, gv, ns, _ = gu.search(idx, Q, k=100, nprobe=24)
    idx.set_tuning()
    ei, ev = oknn.knn_exact(X, np.arange(X.shape[0]), Q, 100, "l2")
    parity.check_all(Q, X, ps.ids, gi, gv, ei, ev, "l2", 100)


def test_recall_monotone_in_target(big_parts):
    X, Q, idx, ps = big_parts
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q, 10, "l2")
    prev_m = None
    prev_r = None
    for tau in (0.5, 0.8, 0.9, 0.95, 0.99, 1.0):
        gi, _, ns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=1.0)
        rec = oknn.recall_at_k(gi, truth, 10)
        if prev_m is not None:
            assert (ns >= prev_m).all()
            assert (rec >= prev_r - 1e-12).all()
        prev_m, prev_r = ns, rec
    assert (prev_r == 1.0).all()


@pytest.mark.parametrize("mode", [dict(recall_target=0.9, f_M=0.5), dict(nprobe=5)])
def test_autotune_picks_knobs_without_changing_results(big_parts, mode):
    X, Q, idx, ps = big_parts
    idx.set_tuning()
    base = gu.search(idx, Q, k=20, **mode)
    knobs, ms = idx.autotune(gu.to_dev(Q), reps=2, k=20, **mode)
    assert ms > 0
    assert knobs["chunk_tiles"] in (0, 8, 16, 32, 64, 128)
    assert knobs["rounds_per_sync"] in (0, 2, 4, 8)
    assert knobs["blocks_per_cu"] in (0, 4, 8, 16)
    got = gu.search(idx, Q, k=20, **mode)
    for a, b in zip(base, got):
        assert (a == b).all(), f"tuning {knobs} changed the result"
    idx.set_tuning()
