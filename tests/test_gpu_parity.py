"""Device search vs the CPU oracle, element by element.

Cases: the 100k x 128 L2 workload with fixed nprobe and with adaptive
scanning; a reduced 768-d inner-product workload with Zipf-sized
partitions; k = 100 and 256; ragged dimensions and partitions, empty and
near-empty partitions, fewer than k reachable results, exact ties, nq = 0;
nprobe = nlist against exact search; batch-composition independence.
"""

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import ivf as oivf
from oracle import knn as oknn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_l2():
    w = synth.get_workload("plain-small-100k-d128")
    X = synth.database(w.spec)
    Q = synth.queries(w.spec, w.nq)
    print(f"[build] {w.name} n={X.shape[0]} d={X.shape[1]} nlist={w.nlist}", flush=True)
    idx = gu.build(X, metric="l2", nlist=w.nlist, kmeans_iters=10, seed=3)
    ps = gu.oracle_view(idx, X)
    yield w, X, Q, idx, ps
    idx.free()


@pytest.fixture(scope="module")
def small_ip():
    base = synth.get_workload("batched-1m-d768-ip")
    spec = synth.MixtureSpec(key=21, n=60_000, d=768, n_components=100, zipf_s=1.1, unit_norm=True)
    X = synth.database(spec)
    Q = synth.queries(spec, 300)
    print(f"[build] reduced {base.name} n={X.shape[0]} nlist=120", flush=True)
    idx = gu.build(X, metric="ip", nlist=120, kmeans_iters=8, seed=5)
    ps = gu.oracle_view(idx, X)
    yield X, Q, idx, ps
    idx.free()


def _boundary_tied(q, C, metric, nprobe):
    vals = oknn.distances(q[None], C, metric)[0]
    key = np.sort(oknn.sort_key(vals, metric))
    if nprobe >= key.shape[0]:
        return False
    a, b = key[nprobe - 1], key[nprobe]
    scale = abs(a) if metric == "l2" else float(np.linalg.norm(q)) * float(np.linalg.norm(C, axis=1).max())
    return abs(b - a) <= 1e-5 * max(scale, 1e-30)


def test_build_places_every_vector_in_its_nearest_partition(small_l2):
    w, X, Q, idx, ps = small_l2
    bad = oivf.assignment_violations(X, ps.assign, ps.C, "l2", rtol=1e-5)
    assert bad.size == 0, f"{bad.size} vectors not in their nearest partition"
    n_live, nparts, _ = idx.stats()
    assert n_live == X.shape[0] and nparts == w.nlist


def test_ip_build_places_every_vector_in_its_best_partition(small_ip):
    X, Q, idx, ps = small_ip
    bad = oivf.assignment_violations(X, ps.assign, ps.C, "ip", rtol=1e-5)
    assert bad.size == 0, f"{bad.size} vectors not in their highest-scoring partition"
    # spherical k-means: unit-length centroids
    np.testing.assert_allclose(np.linalg.norm(ps.C.astype(np.float64), axis=1), 1.0, atol=1e-5)


def test_build_is_reproducible():
    """Cluster sums are exact integers in fixed point, so two builds with one
    seed give bit-identical centroids and the same placement."""
    spec = synth.MixtureSpec(key=23, n=30_000, d=96, n_components=50, zipf_s=1.1, unit_norm=True)
    X = synth.database(spec)
    out = []
    for _ in range(2):
        idx = gu.build(X, metric="ip", nlist=60, kmeans_iters=6, seed=11)
        C, ids, part = idx.export()
        out.append((C.cpu().numpy(), ids.cpu().numpy(), part.cpu().numpy()))
        idx.free()
    (C0, i0, p0), (C1, i1, p1) = out
    assert (C0 == C1).all()
    o0, o1 = np.argsort(i0), np.argsort(i1)
    assert (i0[o0] == i1[o1]).all() and (p0[o0] == p1[o1]).all()


@pytest.mark.parametrize("k", [10, 100, 256])
def test_fixed_nprobe_matches_oracle(small_l2, k):
    w, X, Q, idx, ps = small_l2
    nq = 300 if k > 10 else Q.shape[0]
    Qs = Q[:nq]
    gi, gv, ns, rec = gu.search(idx, Qs, k=k, nprobe=16)
    assert (ns == 16).all() and (rec == 1.0).all()
    ri, rv, _ = oivf.ivf_search(ps, Qs, k, 16, "l2")
    keep = [i for i in range(nq) if not _boundary_tied(Qs[i], ps.C, "l2", 16)]
    assert len(keep) >= 0.99 * nq
    parity.check_all(Qs[keep], X, ps.ids, gi[keep], gv[keep], ri[keep], rv[keep], "l2", k)


def test_all_partitions_equals_exact_search(small_l2):
    w, X, Q, idx, ps = small_l2
    Qs = Q[:100]
    gi, gv, ns, _ = gu.search(idx, Qs, k=10, nprobe=w.nlist)
    ei, ev = oknn.knn_exact(X, np.arange(X.shape[0]), Qs, 10, "l2")
    parity.check_all(Qs, X, ps.ids, gi, gv, ei, ev, "l2", 10)


def _aps_parity(X, Q, idx, ps, metric, f_M, tau_r, k=10):
    gi, gv, ns, rec = gu.search(idx, Q, k=k, recall_target=tau_r, f_M=f_M)
    order, h = idx.candidates(gu.to_dev(Q), f_M)
    parity.check_aps(X, Q, ps, gi, gv, ns, rec, order.cpu().numpy(), h.cpu().numpy(), metric, f_M, tau_r, k)
    return gi, ns


def test_aps_matches_oracle_l2(small_l2):
    w, X, Q, idx, ps = small_l2
    gi, ns = _aps_parity(X, Q, idx, ps, "l2", 0.05, 0.9)
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q, 10, "l2")
    assert oknn.recall_at_k(gi, truth, 10).mean() >= 0.88


@pytest.mark.parametrize("tau", [0.8, 0.95, 0.99])
def test_aps_targets_l2(small_l2, tau):
    w, X, Q, idx, ps = small_l2
    _aps_parity(X, Q[:300], idx, ps, "l2", 0.05, tau)


def test_aps_full_scan_target_one_is_exact(small_l2):
    w, X, Q, idx, ps = small_l2
    Qs = Q[:50]
    gi, gv, ns, rec = gu.search(idx, Qs, k=10, recall_target=1.0, f_M=1.0)
    ei, ev = oknn.knn_exact(X, np.arange(X.shape[0]), Qs, 10, "l2")
    parity.check_all(Qs, X, ps.ids, gi, gv, ei, ev, "l2", 10)


def test_ip_fixed_and_adaptive(small_ip):
    X, Q, idx, ps = small_ip
    gi, gv, ns, _ = gu.search(idx, Q, k=10, nprobe=8)
    ri, rv, _ = oivf.ivf_search(ps, Q, 10, 8, "ip")
    keep = [i for i in range(Q.shape[0]) if not _boundary_tied(Q[i], ps.C, "ip", 8)]
    parity.check_all(Q[keep], X, ps.ids, gi[keep], gv[keep], ri[keep], rv[keep], "ip", 10)
    _aps_parity(X, Q, idx, ps, "ip", 0.1, 0.9)


def test_ip_k100_adaptive(small_ip):
    X, Q, idx, ps = small_ip
    _aps_parity(X, Q[:100], idx, ps, "ip", 0.1, 0.9, k=100)


def test_ragged_dimensions_and_partitions():
    rng = np.random.default_rng(4)
    n, d = 3001, 37
    X = (rng.standard_normal((n, d)) + rng.integers(0, 5, (n, 1))).astype(np.float32)
    ids = rng.permutation(10 * n)[:n].astype(np.int64)
    Q = (X[rng.choice(n, 40, replace=False)] + 0.05 * rng.standard_normal((40, d))).astype(np.float32)
    idx = gu.build(X, ids, metric="l2", nlist=50, kmeans_iters=4, seed=9)
    ps = gu.oracle_view(idx, X, ids)
    for k in (1, 7, 64, 65, 200):
        gi, gv, ns, _ = gu.search(idx, Q, k=k, nprobe=3)
        ri, rv, _ = oivf.ivf_search(ps, Q, k, 3, "l2")
        keep = [i for i in range(Q.shape[0]) if not _boundary_tied(Q[i], ps.C, "l2", 3)]
        parity.check_all(Q[keep], X, ids, gi[keep], gv[keep], ri[keep], rv[keep], "l2", k)
    idx.free()


def test_fewer_results_than_k_and_empty_partitions():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((300, 16)).astype(np.float32)
    C = np.concatenate([X[:5], np.full((3, 16), 50.0, np.float32)])   # 3 centroids nobody is near
    idx = gu.build(X, metric="l2", nlist=8, centroids=gu.to_dev(C))
    ps = gu.oracle_view(idx, X)
    assert (ps.sizes()[5:] == 0).all()
    Q = X[:10] + 0.01
    gi, gv, ns, _ = gu.search(idx, Q, k=256, nprobe=1)
    ri, rv, _ = oivf.ivf_search(ps, Q, 256, 1, "l2")
    parity.check_all(Q, X, ps.ids, gi, gv, ri, rv, "l2", 256)
    assert (gi[:, -1] == -1).all() and np.isinf(gv[:, -1]).all()
    gi, gv, ns, _ = gu.search(idx, Q, k=10, recall_target=0.99, f_M=1.0)
    assert (gi >= 0).all()
    idx.free()


def test_exact_ties_go_to_lower_id():
    rng = np.random.default_rng(8)
    base = rng.standard_normal((40, 8)).astype(np.float32)
    X = np.concatenate([base, base, base])          # every vector three times
    ids = rng.permutation(1000)[:120].astype(np.int64)
    idx = gu.build(X, ids, metric="l2", nlist=4, kmeans_iters=3, seed=2)
    Q = base[:5].copy()
    gi, gv, _, _ = gu.search(idx, Q, k=6, nprobe=4)
    ei, ev = oknn.knn_exact(X, ids, Q, 6, "l2")
    assert (gi == ei).all()
    idx.free()


def test_zero_queries_and_bad_arguments(small_l2):
    from paper_2506_03437_amd import QuakeError
    w, X, Q, idx, ps = small_l2
    torch = gu.torch_mod()
    q0 = torch.empty((0, X.shape[1]), dtype=torch.float32, device="cuda")
    ids, dist, ns, rec = idx.search(q0, k=10, nprobe=4)
    assert ids.shape == (0, 10)
    for kw in ({"k": 0, "nprobe": 4}, {"k": 257, "nprobe": 4}, {"k": 10, "nprobe": 4, "recall_target": 0.9},
               {"k": 10}, {"k": 10, "recall_target": 1.5}):
        with pytest.raises(QuakeError) as e:
            idx.search(gu.to_dev(Q[:2]), **kw)
        assert e.value.code == -1


def test_batch_composition_does_not_change_results(small_l2):
    w, X, Q, idx, ps = small_l2
    a = gu.search(idx, Q[:200], k=10, recall_target=0.9)
    b = gu.search(idx, Q[:200], k=10, recall_target=0.9)
    for x, y in zip(a, b):
        assert (x == y).all()
    alone = gu.search(idx, Q[37:38], k=10, recall_target=0.9)
    mixed = gu.search(idx, np.concatenate([Q[500:600], Q[37:38], Q[600:700]]), k=10, recall_target=0.9)
    for x, y in zip(alone, mixed):
        assert (x[0] == y[100]).all()
