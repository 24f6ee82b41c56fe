"""The C-ABI boundary on the device (Sec. 2.1 problem statement; the build
inputs of Sec. 3): non-finite inputs are rejected before any work, a
caller-given assignment (with or without centroids) places the rows as
given, and index memory comes from the caller's allocator."""

import numpy as np
import pytest

import gpu_util as gu
import synth
from paper_2506_03437_amd import QuakeError, Server, quake

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    spec = synth.MixtureSpec(key=41, n=20_000, d=40, n_components=30, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 200)
    return X, Q


def _invalid(fn):
    with pytest.raises(QuakeError) as e:
        fn()
    assert e.value.code == quake.E_INVALID, e.value
    return str(e.value)


def test_non_finite_inputs_are_rejected(data):
    X, Q = data
    for bad in (np.nan, np.inf, -np.inf):
        Xb = X.copy()
        Xb[1234, 7] = bad
        assert "non-finite" in _invalid(lambda: gu.build(Xb, metric="l2", nlist=32, kmeans_iters=2))
    C = X[:32].copy()
    C[5, 0] = np.inf
    _invalid(lambda: gu.build(X, metric="l2", nlist=32, centroids=gu.to_dev(C)))
    idx = gu.build(X, metric="l2", nlist=32, kmeans_iters=3, seed=2)
    try:
        ref = gu.search(idx, Q, k=10, recall_target=0.9)
        Qb = Q.copy()
        Qb[17, 3] = np.nan
        _invalid(lambda: gu.search(idx, Qb, k=10, recall_target=0.9))
        _invalid(lambda: gu.search(idx, Qb, k=10, nprobe=4, scan_mode="plain"))
        _invalid(lambda: idx.candidates(gu.to_dev(Qb), 0.1))
        # a rejected batch leaves the index as it was
        Xi = X[:50].copy() + 0.5
        Xi[10, 0] = np.inf
        _invalid(lambda: idx.insert(gu.to_dev(Xi), gu.to_dev(np.arange(10**6, 10**6 + 50, dtype=np.int64))))
        assert idx.stats()[0] == X.shape[0]
        again = gu.search(idx, Q, k=10, recall_target=0.9)
        for a, b in zip(ref, again):
            assert (a == b).all()
        with Server(idx, max_slots=64, k=10, recall_target=0.9) as srv:
            _invalid(lambda: srv.search(Qb[15:20]))
            _invalid(lambda: srv.insert(Xi, np.arange(10**6, 10**6 + 50, dtype=np.int64)))
            t = srv.search(Q[:3])
            for i, tk in enumerate(t):
                ids, _, _, st = srv.wait(tk, 60.0)
                assert st == 0 and (ids == ref[0][i]).all()
    finally:
        idx.free()


def test_given_assignment_and_centroids_reproduce_a_build(data):
    """Exporting a build's centroids and placement and building again from
    them gives the same store, hence bit-identical search results."""
    X, Q = data
    idx = gu.build(X, metric="l2", nlist=48, kmeans_iters=5, seed=4)
    try:
        C, ids, part = idx.export()
        assign = np.empty(X.shape[0], dtype=np.int32)
        assign[ids.cpu().numpy()] = part.cpu().numpy()
        ref = gu.search(idx, Q, k=10, recall_target=0.9)
        ref_np = gu.search(idx, Q, k=10, nprobe=6)
    finally:
        idx.free()
    idx2 = gu.build(X, metric="l2", nlist=48, centroids=C.contiguous(), assign=gu.to_dev(assign))
    try:
        C2, ids2, part2 = idx2.export()
        assert (C2.cpu().numpy() == C.cpu().numpy()).all()
        a2 = np.empty(X.shape[0], dtype=np.int32)
        a2[ids2.cpu().numpy()] = part2.cpu().numpy()
        assert (a2 == assign).all()
        for a, b in zip(ref, gu.search(idx2, Q, k=10, recall_target=0.9)):
            assert (a == b).all()
        for a, b in zip(ref_np, gu.search(idx2, Q, k=10, nprobe=6)):
            assert (a == b).all()
    finally:
        idx2.free()


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_assignment_without_centroids_takes_partition_means(metric):
    """Given only the assignment, a centroid is the mean of its rows (unit
    length for inner product); rows stay where the caller put them, even
    where another centroid is nearer."""
    spec = synth.MixtureSpec(key=43, n=6_000, d=24, n_components=12, unit_norm=(metric == "ip"))
    X = synth.database(spec)
    rng = np.random.default_rng(0)
    nlist = 20
    assign = rng.integers(0, nlist, X.shape[0]).astype(np.int32)
    assign[:nlist] = np.arange(nlist)          # every partition gets a row
    idx = gu.build(X, metric=metric, nlist=nlist, assign=gu.to_dev(assign))
    try:
        C, ids, part = idx.export()
        C = C.cpu().numpy()
        got = np.empty(X.shape[0], dtype=np.int32)
        got[ids.cpu().numpy()] = part.cpu().numpy()
        assert (got == assign).all()
        X64 = X.astype(np.float64)
        for j in range(nlist):
            m = X64[assign == j].mean(0)
            if metric == "ip":
                m /= np.linalg.norm(m)
            np.testing.assert_allclose(C[j], m, rtol=0, atol=2e-6 * max(1.0, float(np.abs(m).max())))
    finally:
        idx.free()


def test_bad_assignments_are_rejected(data):
    X, _ = data
    a = np.zeros(X.shape[0], dtype=np.int32)
    a[100] = 16
    assert "outside" in _invalid(lambda: gu.build(X, metric="l2", nlist=16, assign=gu.to_dev(a)))
    a[100] = -1
    _invalid(lambda: gu.build(X, metric="l2", nlist=16, assign=gu.to_dev(a)))
    a = (np.arange(X.shape[0]) % 15).astype(np.int32)   # partition 15 gets nothing
    assert "empty" in _invalid(lambda: gu.build(X, metric="l2", nlist=16, assign=gu.to_dev(a)))


def test_index_memory_comes_from_the_torch_allocator(data):
    import torch
    X, Q = data
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    idx = gu.build(X, metric="l2", nlist=32, kmeans_iters=3, seed=6, storage="bf16")
    try:
        held = idx.stats()[2]
        r_torch = gu.search(idx, Q, k=10, recall_target=0.9)
        r_torch_b = gu.search(idx, Q, k=10, recall_target=0.9, scan_mode="batched", scan_dtype="bf16")
        torch.cuda.synchronize()
        grown = torch.cuda.memory_allocated() - before
        # the store, id map and search workspace are torch allocations
        assert held > 4 * X.nbytes // 2 and grown >= held
    finally:
        idx.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before < held // 10
    idx = gu.build(X, metric="l2", nlist=32, kmeans_iters=3, seed=6, storage="bf16", allocator="hip")
    try:
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - before < held // 10
        for a, b in zip(r_torch, gu.search(idx, Q, k=10, recall_target=0.9)):
            assert (a == b).all()
        for a, b in zip(r_torch_b, gu.search(idx, Q, k=10, recall_target=0.9, scan_mode="batched",
                                             scan_dtype="bf16")):
            assert (a == b).all()
    finally:
        idx.free()


def test_index_without_fp32_tiles(data):
    """drop_f32_tiles: the batched path (16-bit tiles, rerank from the
    row-major FP32 copy) answers bit for bit as with the FP32 tiles, updates
    and maintenance keep working, plain FP32 searches are refused, and the
    index holds a third less memory."""
    X, Q = data
    kw = dict(k=10, recall_target=0.9, scan_mode="batched", scan_dtype="bf16", rerank_factor=4)
    full = gu.build(X, metric="l2", nlist=32, storage="bf16", kmeans_iters=3, seed=2)
    lean = gu.build(X, metric="l2", nlist=32, storage="bf16", kmeans_iters=3, seed=2, f32_tiles=False)
    try:
        assert lean.stats()[2] < 0.75 * full.stats()[2]
        for a, b in zip(gu.search(full, Q, **kw), gu.search(lean, Q, **kw)):
            assert (a == b).all()
        msg = _invalid(lambda: gu.search(lean, Q, k=10, recall_target=0.9))
        assert "FP32 tile" in msg
        rng = np.random.default_rng(8)
        B = (X[rng.choice(X.shape[0], 3000)] + 0.1).astype(np.float32)
        bid = np.arange(10**6, 10**6 + 3000, dtype=np.int64)
        for idx in (full, lean):
            idx.insert(gu.to_dev(B), gu.to_dev(bid))
            idx.delete(gu.to_dev(bid[::2]))
        for a, b in zip(gu.search(full, Q, **kw), gu.search(lean, Q, **kw)):
            assert (a == b).all()
        lam = ([1, 100, 1000, 10000], [1.0, 3.0, 25.0, 300.0])
        hits = np.full(32, 50, dtype=np.int64)
        hits[:4] = 1000
        ra, da = full.maintain(*lam, tau=0.5, hits=hits, window=1000)
        rb, db = lean.maintain(*lam, tau=0.5, hits=hits, window=1000)
        assert ra == rb and da == db and ra["splits"] >= 1
        for a, b in zip(gu.search(full, Q, **kw), gu.search(lean, Q, **kw)):
            assert (a == b).all()
        _invalid(lambda: gu.build(X, metric="l2", nlist=32, storage="f32", f32_tiles=False))
    finally:
        full.free()
        lean.free()
