"""Helpers for the device tests: build through the C ABI, export the
partitioning, and rebuild the same partitioning on the CPU for the oracle."""

from __future__ import annotations

import numpy as np

from oracle import ivf as oivf


def torch_mod():
    import torch
    return torch


def to_dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def build(X, ids=None, **kw):
    from paper_2506_03437_amd import Index
    return Index(to_dev(X), None if ids is None else to_dev(ids), **kw)


def oracle_view(idx, X, ids=None):
    """PartitionedSet with the device index's centroids and assignment."""
    C, eids, epart = idx.export()
    C = C.cpu().numpy()
    eids = eids.cpu().numpy()
    epart = epart.cpu().numpy()
    ids = np.arange(X.shape[0]) if ids is None else np.asarray(ids)
    assert eids.shape[0] == ids.shape[0], "export lost or duplicated vectors"
    row_of = {int(i): r for r, i in enumerate(ids.tolist())}
    assign = np.empty(ids.shape[0], dtype=np.int64)
    seen = np.zeros(ids.shape[0], dtype=bool)
    for i, p in zip(eids.tolist(), epart.tolist()):
        r = row_of[i]
        assert not seen[r], f"id {i} stored twice"
        seen[r] = True
        assign[r] = p
    assert seen.all()
    return oivf.PartitionedSet(X, ids, assign, C)


def search(idx, Q, **kw):
    ids, dist, ns, rec = idx.search(to_dev(Q), **kw)
    torch_mod().cuda.synchronize()
    return ids.cpu().numpy(), dist.cpu().numpy(), ns.cpu().numpy(), rec.cpu().numpy()
