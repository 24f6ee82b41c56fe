"""The 10M x 768 precision workload's code path at reduced size.

Same shape parameters as the full workload except the row count: inner
product on unit-norm 768-d rows from the Zipf(1.1) mixture, 4,096
partitions (so f_M = 0.05 gives M = 205 candidates, past the one-wave
selection: k_select + k_geometry), a BF16 copy with FP32 rerank, and one
16,384-query search call on each path.

* Plain FP32 path: on a seeded sample of the 16,384 queries, results are
  exactly the top-k over the partitions scanned, the candidate order is the
  oracle's Algorithm "Adaptive Partition Scanning" order, and stop counts and
  recall estimates replay the oracle.
* Batched BF16 path: the same candidate order (same kernels), reranked
  distances are the exact FP32 distances of the returned ids, and recall@10
  against FP64 ground truth stays within 0.005 of the FP32 path.
"""

import numpy as np
import pytest

import gpu_util as gu
import parity
import synth
from oracle import knn as oknn

pytestmark = pytest.mark.gpu

NQ = 16_384
F_M = 0.05


@pytest.fixture(scope="module")
def precision_path():
    base = synth.get_workload("precision-10m-d768-bf16")
    spec = synth.MixtureSpec(key=31, n=600_000, d=768, n_components=base.spec.n_components, zipf_s=1.1,
                             unit_norm=True)
    X = synth.database(spec)
    Q = synth.queries(spec, NQ)
    print(f"[build] reduced {base.name}: n={X.shape[0]} nlist={base.nlist} queries={NQ}", flush=True)
    idx = gu.build(X, metric="ip", nlist=base.nlist, storage="bf16", kmeans_iters=4, seed=9)
    ps = gu.oracle_view(idx, X)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(NQ, 128, replace=False))
    yield X, Q, idx, ps, sample
    idx.free()


def test_candidate_count_takes_the_large_selection(precision_path):
    X, Q, idx, ps, sample = precision_path
    order, h = idx.candidates(gu.to_dev(Q[:8]), F_M)
    assert order.shape[1] == 205 and ps.nlist == 4096


@pytest.mark.parametrize("tau", [0.8, 0.9, 0.95])
def test_plain_fp32_matches_oracle(precision_path, tau):
    X, Q, idx, ps, sample = precision_path
    gi, gv, ns, rec = gu.search(idx, Q, k=10, recall_target=tau, f_M=F_M)
    order, h = idx.candidates(gu.to_dev(Q[sample]), F_M)
    parity.check_aps(X, Q, ps, gi, gv, ns, rec, order.cpu().numpy(), h.cpu().numpy(), "ip", F_M, tau, 10,
                     rows=sample)


def test_batched_bf16_path(precision_path):
    X, Q, idx, ps, sample = precision_path
    truth, _ = oknn.knn_exact(X, np.arange(X.shape[0]), Q[sample], 10, "ip")
    id_to_row = {i: i for i in range(X.shape[0])}
    order, h = idx.candidates(gu.to_dev(Q[sample]), F_M)
    order, h = order.cpu().numpy(), h.cpu().numpy()
    for j, i in enumerate(sample[:40].tolist()):
        parity.check_candidate_order(Q[i], ps.C, F_M, "ip", order[j], h[j])
    for tau in (0.8, 0.9, 0.95):
        fi, _, fns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=F_M)
        bi, bv, bns, _ = gu.search(idx, Q, k=10, recall_target=tau, f_M=F_M, scan_mode="batched",
                                   scan_dtype="bf16", rerank_factor=4)
        rf = oknn.recall_at_k(fi[sample], truth, 10).mean()
        rb = oknn.recall_at_k(bi[sample], truth, 10).mean()
        print(f"[recall] tau {tau}: fp32 {rf:.4f} bf16+rerank {rb:.4f} "
              f"(partitions {fns.mean():.2f} / {bns.mean():.2f})", flush=True)
        assert rb >= rf - 0.005, (tau, rf, rb)
        for i in sample[::8].tolist():
            live = bi[i][bi[i] >= 0]
            assert live.size == 10
            tv = parity.true_values(Q[i], X, id_to_row, live, "ip")
            assert (np.abs(bv[i] - tv) <= parity.value_tol(Q[i], X, "ip", tv)).all()
            assert (np.diff(bv[i]) <= 0).all()
