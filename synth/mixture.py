"""Gaussian-mixture vector sets with clustered spatial skew.

The paper's workload generator clusters vectors and samples from the
clusters to create hot spots (Sec. 7.1, "Workload Generator").  The
datasets it measures on are not available, so every workload here is drawn
from a seeded mixture instead:

* component means  mu_c ~ N(0, I_d)                      (stream 0)
* component weights uniform, or w_c proportional to (c+1)^-s (Zipf)
* a database row   x = mu_c + std * z,  c ~ w, z ~ N(0, I_d)  (stream 2)
* inner-product workloads normalise every row to unit length
* a query          a database row plus N(0, noise_std^2) noise, renormalised
  for inner-product workloads                           (stream 3)

Every stream is a PCG64 generator seeded from
``SeedSequence(ENTROPY, spawn_key=(workload_key, stream, chunk))``, so chunks
can be regenerated independently and a 10M-row set never has to be held in
FP64.  Arrays are float32: the database is stored and searched in FP32.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, Optional, Tuple

import numpy as np

ENTROPY = 2506_03437

STREAM_MEANS = 0
STREAM_WEIGHTS = 1
STREAM_DATA = 2
STREAM_QUERIES = 3
STREAM_INIT = 4
STREAM_TRACE = 5
STREAM_LEAVES = 6


def rng_for(key: int, stream: int, chunk: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(ENTROPY, spawn_key=(int(key), int(stream), int(chunk)))
    return np.random.Generator(np.random.PCG64(ss))


@dataclass(frozen=True)
class MixtureSpec:
    key: int                 # workload key: separates the seed streams of workloads
    n: int                   # database rows
    d: int                   # dimension
    n_components: int        # mixture components
    zipf_s: Optional[float] = None   # None: uniform component weights
    comp_std: float = 0.1
    unit_norm: bool = False  # inner-product workloads
    chunk: int = 65536       # rows per independently seeded chunk
    component_offset: int = 0  # first component index (new components for inserts)

    @property
    def n_chunks(self) -> int:
        return (self.n + self.chunk - 1) // self.chunk


def component_means(spec: MixtureSpec, n_total: Optional[int] = None) -> np.ndarray:
    """Means of components [0, n_total) as float64 [n_total, d].

    Components are drawn in a fixed order, so a spec with more components
    (for insert batches from new components) extends the same table.
    """
    c = spec.component_offset + spec.n_components if n_total is None else n_total
    rng = rng_for(spec.key, STREAM_MEANS)
    return rng.standard_normal((c, spec.d))


def component_weights(spec: MixtureSpec) -> np.ndarray:
    c = spec.n_components
    if spec.zipf_s is None:
        w = np.ones(c)
    else:
        w = (np.arange(c, dtype=np.float64) + 1.0) ** (-float(spec.zipf_s))
    return w / w.sum()


def _chunk_raw(spec: MixtureSpec, ci: int, means32: np.ndarray, w: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    lo = ci * spec.chunk
    rows = min(spec.chunk, spec.n - lo)
    rng = rng_for(spec.key, STREAM_DATA, ci)
    comp = rng.choice(spec.n_components, size=rows, p=w) + spec.component_offset
    z = rng.standard_normal((rows, spec.d), dtype=np.float32)
    raw = means32[comp] + np.float32(spec.comp_std) * z
    return comp.astype(np.int32), raw


def _normalise(x: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", x, x, dtype=np.float32))
    return (x / nrm[:, None]).astype(np.float32)


class _Tables:
    def __init__(self, spec: MixtureSpec):
        self.means32 = component_means(spec).astype(np.float32)
        self.w = component_weights(spec)


def database_chunk(spec: MixtureSpec, ci: int, tables: Optional[_Tables] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Rows of chunk ``ci``: (component int32 [rows], x float32 [rows, d])."""
    t = tables or _Tables(spec)
    comp, raw = _chunk_raw(spec, ci, t.means32, t.w)
    return comp, (_normalise(raw) if spec.unit_norm else raw)


def iter_database(spec: MixtureSpec) -> Iterator[Tuple[int, np.ndarray, np.ndarray]]:
    t = _Tables(spec)
    for ci in range(spec.n_chunks):
        comp, x = database_chunk(spec, ci, t)
        yield ci * spec.chunk, comp, x


def database(spec: MixtureSpec, with_components: bool = False):
    """The whole database as float32 [n, d] (and component labels)."""
    x = np.empty((spec.n, spec.d), dtype=np.float32)
    comp = np.empty(spec.n, dtype=np.int32)
    for lo, c, xc in iter_database(spec):
        x[lo:lo + xc.shape[0]] = xc
        comp[lo:lo + xc.shape[0]] = c
    return (x, comp) if with_components else x


def query_rows(spec: MixtureSpec, nq: int, stream_chunk: int = 0) -> np.ndarray:
    """Database rows the queries are drawn around (sampled without replacement)."""
    rng = rng_for(spec.key, STREAM_QUERIES, stream_chunk)
    return np.sort(rng.choice(spec.n, size=nq, replace=False))


def queries(spec: MixtureSpec, nq: int, noise_std: float = 0.1, stream_chunk: int = 0) -> np.ndarray:
    """Queries: database rows plus N(0, noise_std^2) noise, float32 [nq, d].

    Rows are returned in a seeded random order (not sorted by source row).
    For unit-norm workloads the noise is added to the raw row before the
    row is normalised, so that the query stays near its source.
    """
    rows = query_rows(spec, nq, stream_chunk)
    t = _Tables(spec)
    raw = np.empty((nq, spec.d), dtype=np.float32)
    chunk_of = rows // spec.chunk
    for ci in np.unique(chunk_of):
        _, r = _chunk_raw(spec, int(ci), t.means32, t.w)
        sel = np.nonzero(chunk_of == ci)[0]
        raw[sel] = r[rows[sel] - ci * spec.chunk]
    rng = rng_for(spec.key, STREAM_QUERIES, 1_000_000 + stream_chunk)
    noise = rng.standard_normal((nq, spec.d), dtype=np.float32) * np.float32(noise_std)
    perm = rng.permutation(nq)
    q = (raw + noise)[perm]
    return _normalise(q) if spec.unit_norm else q.astype(np.float32)


@dataclass(frozen=True)
class LeafSpec:
    """Database drawn around generator-defined leaves (two-level workloads).

    ``n_leaves`` leaf centres are mixture draws; leaf sizes follow a Zipf law
    over a random ranking of the leaves; a row is its leaf centre plus
    ``leaf_std`` noise.  The leaf a row was drawn from is *not* the partition
    it belongs to: the index assigns rows to their nearest centre itself.
    """
    mixture: MixtureSpec
    n_leaves: int
    leaf_zipf_s: float = 1.1
    leaf_std: float = 0.05
    min_leaf: int = 16
    extra: dict = field(default_factory=dict, compare=False, hash=False)


def leaf_spec_database(ls: LeafSpec):
    """(leaf centres float32 [L, d], leaf-of-row int32 [n], x float32 [n, d])."""
    m = ls.mixture
    t = _Tables(m)
    rng = rng_for(m.key, STREAM_LEAVES, 0)
    comp = rng.choice(m.n_components, size=ls.n_leaves, p=t.w)
    centres = t.means32[comp] + np.float32(m.comp_std) * rng.standard_normal((ls.n_leaves, m.d), dtype=np.float32)
    rank = rng.permutation(ls.n_leaves)
    w = (rank + 1.0) ** (-ls.leaf_zipf_s)
    w = w / w.sum()
    free = m.n - ls.min_leaf * ls.n_leaves
    if free < 0:
        raise ValueError("n too small for min_leaf * n_leaves")
    sizes = ls.min_leaf + np.floor(w * free).astype(np.int64)
    sizes[np.argmax(w)] += m.n - sizes.sum()
    leaf_of = np.repeat(np.arange(ls.n_leaves, dtype=np.int32), sizes)
    leaf_of = leaf_of[rng.permutation(m.n)]
    x = np.empty((m.n, m.d), dtype=np.float32)
    for ci in range(m.n_chunks):
        lo = ci * m.chunk
        hi = min(m.n, lo + m.chunk)
        r = rng_for(m.key, STREAM_DATA, ci)
        z = r.standard_normal((hi - lo, m.d), dtype=np.float32)
        x[lo:hi] = centres[leaf_of[lo:hi]] + np.float32(ls.leaf_std) * z
    if m.unit_norm:
        x = _normalise(x)
    return centres, leaf_of, x
