"""Continuous-batching serving loop (quake_server_*) on the device.

* Each search answers the same alone and in the mix: the ids, distances and
  scanned counts of a query submitted with hundreds of others (admitted into
  free slots while earlier ones are still scanning) equal, bit for bit, those
  of the same query served on its own and those of quake_search.
* With a fixed nprobe the answers also equal the oracle's over the index's
  own partitioning.
* Updates keep submission order: searches queued before an insert see the
  old state, those after it the new one, and a failing update batch reports
  its error without stopping the loop.
* Admission follows the slot limit and the HBM budget.
"""

import threading

import numpy as np
import pytest

import gpu_util as gu
import parity
from oracle import ivf as oivf

pytestmark = pytest.mark.gpu


def _data(n, d, seed, metric="l2", nq=160):
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((24, d)) * 3
    X = (mu[rng.integers(0, 24, n)] + rng.standard_normal((n, d))).astype(np.float32)
    Q = (mu[rng.integers(0, 24, nq)] + rng.standard_normal((nq, d))).astype(np.float32)
    if metric == "ip":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return X, Q, rng, mu


def _serve_all(srv, Q):
    tickets = srv.search(Q)
    out = [srv.wait(t, timeout_s=60.0) for t in tickets]
    assert all(o[3] == 0 for o in out)
    return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]), np.array([o[2] for o in out]))


def _serve_alone(srv, Q):
    out = []
    for q in Q:
        (t,) = srv.search(q[None, :])
        out.append(srv.wait(t, timeout_s=60.0))
    return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]), np.array([o[2] for o in out]))


def _same(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert (x == y).all()


CASES = [
    ("l2", "f32", dict(k=10, recall_target=0.9, f_M=0.25)),
    ("l2", "f32", dict(k=10, nprobe=5)),
    ("ip", "bf16", dict(k=10, recall_target=0.9, f_M=0.25, scan_mode="batched", scan_dtype="bf16")),
    ("l2", "f16", dict(k=16, recall_target=0.95, f_M=0.3, scan_mode="batched", scan_dtype="f16")),
]


@pytest.mark.parametrize("metric,storage,kw", CASES)
def test_alone_equals_mix_equals_search(metric, storage, kw):
    from paper_2506_03437_amd import Server
    X, Q, _, _ = _data(12_000, 48, 7, metric)
    print(f"[case] {metric} {storage} {kw}", flush=True)
    idx = gu.build(X, metric=metric, nlist=48, storage=storage, kmeans_iters=4, seed=3)
    try:
        ref = gu.search(idx, Q, **kw)[:3]
        with Server(idx, max_slots=24, **kw) as srv:
            mix = _serve_all(srv, Q)
            rounds_mix = srv.stats(reset=True)["rounds"]
            alone = _serve_alone(srv, Q[:40])
            rounds_alone = srv.stats()["rounds"]
        _same(mix, ref)
        _same(alone, tuple(r[:40] for r in ref))
        # in the mix the searches share rounds
        assert rounds_mix < rounds_alone * Q.shape[0] / 40
        if "nprobe" in kw:
            ps = gu.oracle_view(idx, X)
            ri, rv, _ = oivf.ivf_search(ps, Q, kw["k"], kw["nprobe"], metric)
            parity.check_all(Q, ps.X, ps.ids, mix[0], mix[1], ri, rv, metric, kw["k"])
    finally:
        idx.free()


def test_arrivals_while_searches_run():
    """Queries submitted from another thread in small bursts join the running batch."""
    from paper_2506_03437_amd import Server
    X, Q, _, _ = _data(20_000, 32, 11, nq=300)
    kw = dict(k=10, recall_target=0.92, f_M=0.2)
    idx = gu.build(X, nlist=64, kmeans_iters=4, seed=5)
    try:
        ref = gu.search(idx, Q, **kw)[:3]
        with Server(idx, max_slots=32, **kw) as srv:
            tickets = [None] * Q.shape[0]

            def producer():
                for s in range(0, Q.shape[0], 7):
                    first = srv.search(Q[s:s + 7])
                    tickets[s:s + len(first)] = first

            th = threading.Thread(target=producer)
            th.start()
            th.join()
            out = [srv.wait(t, timeout_s=60.0) for t in tickets]
            st = srv.stats()
        got = (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]), np.array([o[2] for o in out]))
        _same(got, ref)
        assert st["completed"] == Q.shape[0]
        assert 1 <= st["max_in_flight"] <= st["slots"] == 32
        assert st["in_flight"] == 0 and st["queued"] == 0
        assert 0 < st["p50_latency_s"] <= st["p99_latency_s"] and st["qps"] > 0
    finally:
        idx.free()


def test_updates_keep_submission_order():
    from paper_2506_03437_amd import QuakeError, Server
    X, Q, rng, mu = _data(10_000, 32, 13, nq=80)
    kw = dict(k=10, recall_target=0.9, f_M=0.3)
    idx = gu.build(X, nlist=40, kmeans_iters=4, seed=2)
    B = (mu[rng.integers(0, 24, 3000)] + rng.standard_normal((3000, 32))).astype(np.float32)
    bid = np.arange(50_000, 53_000, dtype=np.int64)
    try:
        r0 = gu.search(idx, Q, **kw)[:3]
        with Server(idx, max_slots=16, **kw) as srv:
            ta = srv.search(Q)
            ti = srv.insert(B, bid)
            tdup = srv.insert(B[:2], np.array([7, 7], dtype=np.int64))  # duplicate ids: rejected
            tc = srv.search(Q)
            td = srv.delete(bid)
            te = srv.search(Q)
            res = {}
            for name, ts in (("a", ta), ("c", tc), ("e", te)):
                out = [srv.wait(t, timeout_s=60.0) for t in ts]
                res[name] = (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]),
                             np.array([o[2] for o in out]))
            assert srv.wait(ti, timeout_s=60.0)[3] == 0
            assert srv.wait(tdup, timeout_s=60.0)[3] == -4
            assert srv.wait(td, timeout_s=60.0)[3] == 0
            assert srv.stats()["epochs"] == 3
        assert idx.stats()[0] == X.shape[0]
        idx.insert(gu.to_dev(B), gu.to_dev(bid))
        r1 = gu.search(idx, Q, **kw)[:3]
        idx.delete(gu.to_dev(bid))
        _same(res["a"], r0)
        _same(res["c"], r1)
        _same(res["e"], r0)
        assert not all((x == y).all() for x, y in zip(r0, r1))
        with pytest.raises(QuakeError):
            Server(idx, k=10, nprobe=0, recall_target=0.0)  # neither nprobe nor a recall target
    finally:
        idx.free()


def test_hbm_budget_limits_slots():
    from paper_2506_03437_amd import QuakeError, Server
    X, Q, _, _ = _data(8_000, 32, 17, nq=50)
    kw = dict(k=10, nprobe=4)
    idx = gu.build(X, nlist=32, kmeans_iters=3, seed=4)
    try:
        ref = gu.search(idx, Q, **kw)[:3]
        with pytest.raises(QuakeError) as e:
            Server(idx, hbm_budget_bytes=64, **kw)
        assert e.value.code == -2
        with Server(idx, hbm_budget_bytes=6 * 4096, **kw) as srv:
            slots = srv.stats()["slots"]
            got = _serve_all(srv, Q)
            st = srv.stats()
        assert 1 <= slots < 50
        assert st["max_in_flight"] <= slots
        _same(got, ref)
    finally:
        idx.free()


@pytest.mark.parametrize("batched", [False, True])
def test_overlapped_updates_keep_submission_order(batched):
    """With overlap_updates the server applies an update beside the searches
    admitted before it (on a second copy of the store); every search still
    answers, bit for bit, as on the index state of its epoch."""
    from paper_2506_03437_amd import Server
    X, Q, rng, mu = _data(10_000, 32, 19, nq=120)
    kw = dict(k=10, recall_target=0.99, f_M=0.3)
    storage = "bf16" if batched else "f32"
    if batched:
        kw.update(scan_mode="batched", scan_dtype="bf16", rerank_factor=4)
    build = dict(nlist=40, storage=storage, kmeans_iters=4, seed=2)
    B = (mu[rng.integers(0, 24, 3000)] + rng.standard_normal((3000, 32))).astype(np.float32)
    bid = np.arange(60_000, 63_000, dtype=np.int64)
    idx = gu.build(X, **build)
    ref = gu.build(X, **build)  # builds are bit-reproducible
    try:
        r0 = gu.search(idx, Q, **kw)[:3]
        ref.insert(gu.to_dev(B), gu.to_dev(bid))
        r1 = gu.search(ref, Q, **kw)[:3]
        with Server(idx, max_slots=64, overlap_updates=True, **kw) as srv:
            ta = srv.search(Q)
            ti = srv.insert(B, bid)
            tc = srv.search(Q)
            td = srv.delete(bid)
            te = srv.search(Q)
            tdup = srv.insert(B[:2], np.array([7, 7], dtype=np.int64))  # rejected: the versions stay equal
            tf = srv.search(Q)
            res = {}
            for name, ts in (("a", ta), ("c", tc), ("e", te), ("f", tf)):
                out = [srv.wait(t, timeout_s=60.0) for t in ts]
                assert all(o[3] == 0 for o in out)
                res[name] = (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]),
                             np.array([o[2] for o in out]))
            assert srv.wait(ti, timeout_s=60.0)[3] == 0
            assert srv.wait(td, timeout_s=60.0)[3] == 0
            assert srv.wait(tdup, timeout_s=60.0)[3] == -4
            st = srv.stats()
        print(f"[serving] {st}", flush=True)
        assert st["epochs"] == 3 and st["overlapped_updates"] >= 1
        assert idx.stats()[0] == X.shape[0]
        r2 = gu.search(idx, Q, **kw)[:3]  # the index now holds the newest version
        _same(res["a"], r0)
        _same(res["c"], r1)
        _same(res["e"], r2)
        _same(res["f"], r2)
        assert not all((x == y).all() for x, y in zip(r0, r1))
    finally:
        idx.free()
        ref.free()
