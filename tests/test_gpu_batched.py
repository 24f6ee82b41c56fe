"""Batched reduced-precision scan (queries grouped per partition, BF16/FP16
MFMA scores, FP32 rerank) against the oracle.

* Integer-valued vectors (|x_i| <= 4) are exact in BF16 and FP16 and their
  products and sums are exact in FP32, so on such data the batched path must
  return exactly the oracle's top-k over the partitions it scanned, for L2
  and inner product, fixed nprobe and adaptive scanning, and several
  schedules.
* On the float workloads the FP32 rerank must report exact FP32 distances,
  and recall@10 must stay within 0.005 of the plain FP32 path.
"""

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import aps as oaps
from oracle import ivf as oivf
from oracle import knn as oknn

pytestmark = pytest.mark.gpu


def _int_data(n, d, seed, metric):
    rng = np.random.default_rng(seed)
    centres = rng.integers(-3, 4, (12, d))
    X = centres[rng.integers(0, 12, n)] + rng.integers(-1, 2, (n, d))
    X = np.clip(X, -4, 4).astype(np.float32)
    Q = (centres[rng.integers(0, 12, 256)] + rng.integers(-1, 2, (256, d))).astype(np.float32)
    return X, Q


@pytest.fixture(scope="module", params=[("l2", "bf16"), ("ip", "bf16"), ("l2", "f16")])
def int_index(request):
    metric, dtype = request.param
    X, Q = _int_data(20_000, 64, 3, metric)
    print(f"[build] integer data {metric} {dtype}", flush=True)
    idx = gu.build(X, metric=metric, nlist=40, storage=dtype, kmeans_iters=4, seed=2)
    ps = gu.oracle_view(idx, X)
    yield metric, dtype, X, Q, idx, ps
    idx.free()


def test_batched_exact_on_integer_data_nprobe(int_index):
    metric, dtype, X, Q, idx, ps = int_index
    for k, rf in ((10, 4), (1, 64), (16, 4), (32, 2)):
        gi, gv, ns, _ = gu.search(idx, Q, k=k, nprobe=5, scan_mode="batched", scan_dtype=dtype, rerank_factor=rf)
        assert (ns == 5).all()
        ri, rv, probes = oivf.ivf_search(ps, Q, k, 5, metric)
        parity.check_all(Q, X, ps.ids, gi, gv, ri, rv, metric, k)


@pytest.mark.parametrize("tau", [0.8, 0.9, 0.97])
def test_batched_exact_on_integer_data_aps(int_index, tau):
    """Scores are exact here, so the batched path's adaptive decisions must
    replay the oracle's Algorithm "Adaptive Partition Scanning" query by
    query: the same stop count and recall estimate (up to decisions within
    the floating-point margin of the device's FP32 bisector distances), and
    exactly the top-k over the partitions scanned."""
    metric, dtype, X, Q, idx, ps = int_index
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=tau, f_M=0.3, scan_mode="batched", scan_dtype=dtype)
    order, h = idx.candidates(gu.to_dev(Q), 0.3)
    parity.check_aps(X, Q, ps, gi, gv, ns, rec, order.cpu().numpy(), h.cpu().numpy(), metric, 0.3, tau, 10)
    # the plain FP32 path takes the same decisions on this data
    fi, fv, fns, frec = gu.search(idx, Q, k=10, recall_target=tau, f_M=0.3)
    assert (fns == ns).all() and (fi == gi).all()


def test_batched_schedules_agree(int_index):
    metric, dtype, X, Q, idx, ps = int_index
    kw = dict(k=10, recall_target=0.95, f_M=0.5, scan_mode="batched", scan_dtype=dtype)
    base = gu.search(idx, Q, **kw)
    for sch in (dict(chunk_tiles=1), dict(max_items=1), dict(first_window=1, max_window=1), dict(first_window=16),
                dict(rounds_per_sync=1, blocks_per_cu=1), dict(rounds_per_sync=16, blocks_per_cu=8)):
        idx.set_tuning(**sch)
        got = gu.search(idx, Q, **kw)
        for a, b in zip(base, got):
            assert (a == b).all(), f"schedule {sch} changed the result"
    idx.set_tuning()


@pytest.fixture(scope="module")
def float_ip():
    spec = synth.MixtureSpec(key=22, n=80_000, d=768, n_components=120, zipf_s=1.1, unit_norm=True)
    X = synth.database(spec)
    Q = synth.queries(spec, 500)
    print("[build] 80k x 768 IP with a BF16 copy", flush=True)
    idx = gu.build(X, metric="ip", nlist=160, storage="bf16", kmeans_iters=6, seed=6)
    ps = gu.oracle_view(idx, X)
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q, 10, "ip")
    yield X, Q, idx, ps, truth
    idx.free()


@pytest.mark.parametrize("tau", [0.8, 0.9, 0.95])
def test_bf16_rerank_recall_gap(float_ip, tau):
    X, Q, idx, ps, truth = float_ip
    fi, fv, fns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=0.1)
    bi, bv, bns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=0.1, scan_mode="batched", scan_dtype="bf16")
    rf = oknn.recall_at_k(fi, truth, 10).mean()
    rb = oknn.recall_at_k(bi, truth, 10).mean()
    assert rb >= rf - 0.005, (rf, rb)
    # reported distances are exact FP32 distances of the returned ids
    id_to_row = {i: i for i in range(X.shape[0])}
    for i in range(0, Q.shape[0], 25):
        live = bi[i][bi[i] >= 0]
        tv = parity.true_values(Q[i], X, id_to_row, live, "ip")
        tol = parity.value_tol(Q[i], X, "ip", tv)
        assert (np.abs(bv[i][: live.size] - tv) <= tol).all()


def test_bf16_nprobe_matches_fp32_candidates_closely(float_ip):
    X, Q, idx, ps, truth = float_ip
    fi, fv, _, _ = gu.search(idx, Q, k=10, nprobe=8)
    bi, bv, _, _ = gu.search(idx, Q, k=10, nprobe=8, scan_mode="batched", scan_dtype="bf16", rerank_factor=4)
    same = np.mean([len(set(a.tolist()) & set(b.tolist())) / 10.0 for a, b in zip(fi, bi)])
    assert same >= 0.995, same
    # the rerank sums in the plain scan's order: identical FP32 distances per id
    for a_i, a_v, b_i, b_v in zip(fi, fv, bi, bv):
        da = dict(zip(a_i.tolist(), a_v.tolist()))
        for i, v in zip(b_i.tolist(), b_v.tolist()):
            if i in da:
                assert da[i] == v


def _bf16(a):
    """Round to BF16 (nearest, ties to even), returned as float32 values."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_mfma_scores_within_the_accumulation_bound(float_ip):
    """Without the FP32 rerank the batched path returns its own BF16 MFMA
    scores.  BF16 x BF16 products are exact in FP32, so only the FP32
    accumulation rounds: each score lies within gamma_d * sum |q~_i x~_i|
    (gamma_d = d u / (1 - d u), u = 2^-24) of the FP64 dot product of the
    rounded query and row; and the ids are the top-k of the probed
    partitions by that exact dot, up to values within twice the bound."""
    X, Q, idx, ps, truth = float_ip
    Qs = Q[:120]
    bi, bv, _, _ = gu.search(idx, Qs, k=10, nprobe=8, scan_mode="batched", scan_dtype="bf16", rerank_factor=-1)
    d = X.shape[1]
    u = 2.0 ** -24
    gamma = d * u / (1 - d * u)
    Q16 = _bf16(Qs).astype(np.float64)
    X16 = _bf16(X).astype(np.float64)
    for i in range(Qs.shape[0]):
        _, probes = oivf.centroid_ranking(Qs[i], ps.C, "ip")
        rows = np.concatenate([ps.members[p] for p in probes[:8]])
        exact = X16[rows] @ Q16[i]
        bound = gamma * (np.abs(X16[rows]) @ np.abs(Q16[i]))
        pos = {int(ps.ids[r]): j for j, r in enumerate(rows)}
        got = [pos[int(g)] for g in bi[i]]
        err = np.abs(bv[i].astype(np.float64) - exact[got])
        assert (err <= bound[got]).all(), (i, float((err - bound[got]).max()))
        kth = np.sort(exact)[::-1][9]
        tol = 2 * float(bound.max())
        assert (exact[got] >= kth - tol).all()
        clear = set(np.nonzero(exact > kth + tol)[0].tolist())
        assert clear <= set(got), f"query {i}: a clear top-10 row is missing"


def test_batched_rejects_bad_modes(float_ip):
    from paper_2506_03437_amd import QuakeError
    X, Q, idx, ps, truth = float_ip
    for kw in (dict(scan_mode="batched"), dict(scan_dtype="bf16"), dict(scan_mode="batched", scan_dtype="f16"),
               dict(scan_mode="batched", scan_dtype="bf16", k=20, rerank_factor=4)):
        args = dict(k=10, nprobe=4)
        args.update(kw)
        with pytest.raises(QuakeError):
            idx.search(gu.to_dev(Q[:4]), **args)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_batched_heavy_ties(metric):
    """Every vector stored 20 times: pools fill with equal keys, so cuts land
    inside runs of ties (the slot bisection) and later candidates tie the
    threshold.  Ids are exact on this integer data; ties go to the lower id
    (the 20 copies of a vector all fit in the rerank_factor * k candidates)."""
    rng = np.random.default_rng(21)
    base = rng.integers(-4, 5, (60, 32)).astype(np.float32)
    X = np.repeat(base, 20, axis=0)
    ids = rng.permutation(100_000)[: X.shape[0]].astype(np.int64)
    print(f"[build] heavy ties {metric}", flush=True)
    idx = gu.build(X, ids, metric=metric, nlist=4, storage="bf16", kmeans_iters=3, seed=2)
    try:
        Q = np.clip(base[:16] + rng.integers(-1, 2, (16, 32)), -4, 4).astype(np.float32)
        for k in (10, 16):
            gi, gv, _, _ = gu.search(idx, Q, k=k, nprobe=4, scan_mode="batched", scan_dtype="bf16",
                                     rerank_factor=4)
            ei, ev = oknn.knn_exact(X, ids, Q, k, metric)
            assert (gi == ei).all()
            parity.check_all(Q, X, ids, gi, gv, ei, ev, metric, k)
    finally:
        idx.free()
