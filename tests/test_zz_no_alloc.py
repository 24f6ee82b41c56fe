"""quake_search_noalloc against quake_search: the same results, bit for bit,
on two calls in a row (the second with fewer queries, so it runs on what the
first left in the shared scratch array), with no device allocation during
the call; oversized calls and two-level indexes are refused."""

import gc

import numpy as np
import pytest

import gpu_util as gu
import synth
from paper_2506_03437_amd import QuakeError, quake

pytestmark = pytest.mark.gpu


def _outputs(nq, k):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.full((nq, k), -7, dtype=torch.int64, device=dev),
            torch.full((nq, k), 7.0, dtype=torch.float32, device=dev),
            torch.full((nq,), -7, dtype=torch.int32, device=dev),
            torch.full((nq,), 7.0, dtype=torch.float64, device=dev))


@pytest.fixture(scope="module")
def index():
    spec = synth.MixtureSpec(key=51, n=30_000, d=64, n_components=40, zipf_s=1.1)
    X = synth.database(spec)
    Q = synth.queries(spec, 700)
    print("[build] no-alloc index 30k x 64, 64 partitions, BF16 copy", flush=True)
    idx = gu.build(X, metric="l2", nlist=64, storage="bf16", kmeans_iters=4, seed=3)
    yield idx, Q
    idx.free()


@pytest.mark.parametrize("kw", [dict(k=10, recall_target=0.9, f_M=0.2),
                                dict(k=10, nprobe=6),
                                dict(k=10, recall_target=0.95, f_M=0.2, scan_mode="batched", scan_dtype="bf16"),
                                dict(k=5, nprobe=8, scan_mode="batched", scan_dtype="bf16", rerank_factor=6)])
def test_noalloc_matches_search_on_two_calls(index, kw):
    import torch
    idx, Q = index
    for rows in (slice(0, 500), slice(500, 650)):
        Qd = gu.to_dev(Q[rows])
        ref = [t.cpu().numpy() for t in idx.search(Qd, **kw)]
        out = _outputs(Qd.shape[0], kw["k"])
        gc.collect()
        torch.cuda.synchronize()
        # the caching allocator's count of allocation requests (frees of
        # objects collected meanwhile do not move it)
        before = torch.cuda.memory_stats()["allocation.all.allocated"]
        quake.quake_search_noalloc(idx.handle, Qd, outputs=out, **kw)
        torch.cuda.synchronize()
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
        got = [t.cpu().numpy() for t in out]
        for a, b in zip(ref, got):
            assert a.shape == b.shape and (a == b).all()


def test_noalloc_refuses_what_does_not_fit(index):
    import torch
    idx, _ = index
    big = torch.zeros((600_000, 64), dtype=torch.float32, device=torch.device("cuda", 0))
    with pytest.raises(QuakeError) as e:
        quake.quake_search_noalloc(idx.handle, big, outputs=_outputs(600_000, 10), k=10, nprobe=4)
    assert e.value.code == quake.E_INVALID and "scratch" in str(e.value)


def test_noalloc_refuses_two_level_indexes():
    spec = synth.MixtureSpec(key=52, n=8_000, d=16, n_components=10)
    X = synth.database(spec)
    idx = gu.build(X, metric="l2", nlist=32, n_levels=2, nlist_top=4, kmeans_iters=3)
    try:
        Qd = gu.to_dev(X[:10])
        with pytest.raises(QuakeError) as e:
            quake.quake_search_noalloc(idx.handle, Qd, outputs=_outputs(10, 10), k=10, nprobe=2)
        assert e.value.code == quake.E_STATE
    finally:
        idx.free()
