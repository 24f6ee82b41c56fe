"""Request traces for the serving loop: skewed, drifting queries interleaved
with insert and delete batches.

* Query components follow Zipf(s) over a popularity ranking of the mixture's
  components; the ranking is re-drawn every ``drift_every`` requests, so the
  popular set drifts (the paper's workload generator samples clusters to
  create hot spots and shifts them over time, Sec. 7.1).
* A query is a fresh draw of its component (mean + comp_std * z) plus
  N(0, noise_std^2) noise, renormalised for inner-product workloads.
* After every ``update_every`` queries: one insert batch of
  ``update_frac * n_live`` vectors drawn from ``new_components`` components
  that the database did not have, with fresh ids, then one delete batch of
  as many ids drawn uniformly from the live set.

Everything is drawn from seeded streams (stream 5 of the workload key);
nothing here computes distances or touches the index.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from .mixture import STREAM_TRACE, MixtureSpec, component_means, rng_for


@dataclass(frozen=True)
class TraceSpec:
    n_requests: int = 20_000
    zipf_s: float = 1.2
    drift_every: int = 100_000
    update_every: int = 100_000
    update_frac: float = 0.01
    new_components: int = 10
    noise_std: float = 0.1


def _normalise(x: np.ndarray) -> np.ndarray:
    return (x / np.sqrt((x.astype(np.float64) ** 2).sum(1, keepdims=True))).astype(np.float32)


def serving_trace(spec: MixtureSpec, live_ids: np.ndarray, ts: TraceSpec) -> List[Tuple]:
    """Events in arrival order: ("search", Q [b, d]), ("insert", X [b, d], ids [b])
    and ("delete", ids [b]).  Consecutive queries come as one block."""
    rng = rng_for(spec.key, STREAM_TRACE)
    C = spec.n_components
    n_new_total = (ts.n_requests // max(ts.update_every, 1) + 1) * ts.new_components
    means = component_means(spec, spec.component_offset + C + n_new_total).astype(np.float32)
    ranks = (np.arange(C, dtype=np.float64) + 1.0) ** (-ts.zipf_s)
    ranks /= ranks.sum()
    live = np.asarray(live_ids, dtype=np.int64).copy()
    next_id = int(live.max(initial=-1)) + 1
    perm = rng.permutation(C)
    events: List[Tuple] = []
    done = 0
    epoch = 0
    while done < ts.n_requests:
        # queries up to the next drift or update boundary
        to_drift = ts.drift_every - done % ts.drift_every
        to_update = ts.update_every - done % ts.update_every
        b = min(to_drift, to_update, ts.n_requests - done)
        comp = perm[rng.choice(C, size=b, p=ranks)] + spec.component_offset
        raw = means[comp] + np.float32(spec.comp_std) * rng.standard_normal((b, spec.d), dtype=np.float32)
        if spec.unit_norm:
            raw = _normalise(raw)
        q = raw + np.float32(ts.noise_std) * rng.standard_normal((b, spec.d), dtype=np.float32)
        events.append(("search", _normalise(q) if spec.unit_norm else q.astype(np.float32)))
        done += b
        if done % ts.drift_every == 0:
            perm = rng.permutation(C)
        if done % ts.update_every == 0 and done < ts.n_requests:
            nb = max(1, int(round(ts.update_frac * live.size)))
            first = spec.component_offset + C + epoch * ts.new_components
            comp = first + rng.integers(0, ts.new_components, nb)
            x = means[comp] + np.float32(spec.comp_std) * rng.standard_normal((nb, spec.d), dtype=np.float32)
            if spec.unit_norm:
                x = _normalise(x)
            ids = np.arange(next_id, next_id + nb, dtype=np.int64)
            next_id += nb
            events.append(("insert", x.astype(np.float32), ids))
            live = np.concatenate([live, ids])
            pick = rng.choice(live.size, size=nb, replace=False)
            events.append(("delete", live[pick].copy()))
            live = np.delete(live, pick)
            epoch += 1
    return events
