"""Seeded label bits for filtered searches.

Each row carries one of `n_labels` labels as a one-hot 32-bit mask.  Labels
follow location: a row takes its mixture component's home label
(component mod n_labels) with probability `home_prob`, else a label drawn
uniformly, so that partitions differ in how many of their rows pass a
filter.  A query's mask is one label drawn uniformly.
"""

from __future__ import annotations

import numpy as np

from .mixture import MixtureSpec, rng_for

STREAM_LABELS = 7
STREAM_MASKS = 8


def row_labels(spec: MixtureSpec, components: np.ndarray, n_labels: int = 8, home_prob: float = 0.7) -> np.ndarray:
    """uint32 [n] one-hot label masks of the rows with the given components."""
    assert 1 <= n_labels <= 32
    rng = rng_for(spec.key, STREAM_LABELS)
    home = np.asarray(components, dtype=np.int64) % n_labels
    other = rng.integers(0, n_labels, home.shape[0])
    lab = np.where(rng.random(home.shape[0]) < home_prob, home, other)
    return (np.uint32(1) << lab.astype(np.uint32)).astype(np.uint32)


def query_masks(spec: MixtureSpec, nq: int, n_labels: int = 8) -> np.ndarray:
    """uint32 [nq] one-hot masks, one label per query drawn uniformly."""
    rng = rng_for(spec.key, STREAM_MASKS)
    return (np.uint32(1) << rng.integers(0, n_labels, nq).astype(np.uint32)).astype(np.uint32)
