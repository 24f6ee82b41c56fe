"""The named synthetic workloads (shapes, value distributions, search knobs).

Each entry fixes the mixture that generates the database and queries and the
search parameters the workload is run with.  The sizes follow the paper's
workloads in spirit (clustered, skewed, 10^5..10^7 rows, d = 128 or 768);
the datasets themselves are not used.
"""

from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Dict, Optional

from .mixture import LeafSpec, MixtureSpec


@dataclass(frozen=True)
class Workload:
    name: str
    spec: MixtureSpec
    nlist: int
    metric: str                 # "l2" or "ip"
    nq: int
    k: int = 10
    nprobe: int = 0             # > 0: fixed-nprobe search
    recall_target: float = 0.0  # > 0: adaptive partition scanning
    f_M: float = 0.05
    storage: str = "f32"        # extra reduced-precision store copy: f32 | bf16 | f16
    leaves: Optional[LeafSpec] = None
    nlist_top: int = 0
    query_noise: float = 0.1

    def scaled(self, n: int, nq: int, nlist: Optional[int] = None, **kw) -> "Workload":
        spec = replace(self.spec, n=n)
        return replace(self, spec=spec, nq=nq, nlist=nlist or self.nlist, **kw)


WORKLOADS: Dict[str, Workload] = {
    # 100k x 128 FP32, 100 equal components, 256 partitions, L2, nprobe 16.
    "plain-small-100k-d128": Workload(
        name="plain-small-100k-d128",
        spec=MixtureSpec(key=1, n=100_000, d=128, n_components=100),
        nlist=256, metric="l2", nq=1000, k=10, nprobe=16),
    # 1M x 768 unit-norm, 1,000 Zipf(1.1) components, 1,000 partitions, IP,
    # 10,000 queries, recall target 0.9.
    "batched-1m-d768-ip": Workload(
        name="batched-1m-d768-ip",
        spec=MixtureSpec(key=2, n=1_000_000, d=768, n_components=1000, zipf_s=1.1, unit_norm=True),
        nlist=1000, metric="ip", nq=10_000, k=10, recall_target=0.9, f_M=0.05, storage="bf16"),
    # 10M x 768 BF16 store (+FP32 copy for the rerank), 4,096 partitions, IP.
    "precision-10m-d768-bf16": Workload(
        name="precision-10m-d768-bf16",
        spec=MixtureSpec(key=3, n=10_000_000, d=768, n_components=1000, zipf_s=1.1, unit_norm=True),
        nlist=4096, metric="ip", nq=16_384, k=10, recall_target=0.9, f_M=0.05, storage="bf16"),
    # 50M x 128 FP16 store, 50k generator-defined leaves under 64 top partitions, L2.
    # Leaf sizes Zipf(0.3) over a random ranking (mean 1,000, largest about
    # 43k); rows spread 0.2 per dimension around their leaf centre, twice the
    # spread of the centres around their component, so that a query's ten
    # nearest neighbours lie in about six leaves (half in its nearest one).
    "two-level-50m-d128-f16": Workload(
        name="two-level-50m-d128-f16",
        spec=MixtureSpec(key=4, n=50_000_000, d=128, n_components=1000, zipf_s=1.1),
        nlist=50_000, metric="l2", nq=65_536, k=10, recall_target=0.9, f_M=0.015,
        storage="f16", leaves=LeafSpec(MixtureSpec(key=4, n=50_000_000, d=128, n_components=1000, zipf_s=1.1), 50_000,
                                       leaf_zipf_s=0.3, leaf_std=0.2),
        nlist_top=64, query_noise=0.1),
    # Estimator and early-termination ablations: 1M x 128 (the size of the
    # paper's ablation dataset), 1,000 Zipf(1.1) components, 1,000
    # partitions, L2, 10,000 queries, FP16 copy for the batched path.
    "ablation-1m-d128-l2": Workload(
        name="ablation-1m-d128-l2",
        spec=MixtureSpec(key=6, n=1_000_000, d=128, n_components=1000, zipf_s=1.1),
        nlist=1000, metric="l2", nq=10_000, k=10, recall_target=0.9, f_M=0.05, storage="f16"),
    # Levels: 10M x 128, 1,000 Zipf(1.1) components, 40,000 partitions (the
    # partition count of the paper's two-level table), L2, 10,000 queries,
    # f_M 1.5% (600 level-0 candidates), FP16 copy.
    "levels-10m-d128-l2": Workload(
        name="levels-10m-d128-l2",
        spec=MixtureSpec(key=7, n=10_000_000, d=128, n_components=1000, zipf_s=1.1),
        nlist=40_000, metric="l2", nq=10_000, k=10, recall_target=0.9, f_M=0.015, storage="f16"),
    # Serving: 10M x 768 BF16 start, skewed drifting queries, 1% updates per step.
    "serving-10m-d768-bf16": Workload(
        name="serving-10m-d768-bf16",
        spec=MixtureSpec(key=5, n=10_000_000, d=768, n_components=1000, zipf_s=1.1, unit_norm=True),
        nlist=4096, metric="ip", nq=16_384, k=10, recall_target=0.9, f_M=0.05, storage="bf16"),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]
