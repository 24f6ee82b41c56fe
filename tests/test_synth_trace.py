"""The serving trace generator: request counts, update batches with fresh
ids from new components, deletes of live ids only, Zipf skew and drift."""

import numpy as np

import synth


def _spec():
    return synth.MixtureSpec(key=90, n=5_000, d=16, n_components=50, zipf_s=1.1, unit_norm=True)


def test_trace_structure():
    spec = _spec()
    live = np.arange(spec.n, dtype=np.int64)
    ts = synth.TraceSpec(n_requests=2_500, drift_every=1_000, update_every=600, update_frac=0.02, new_components=3)
    ev = synth.serving_trace(spec, live, ts)
    nq = sum(e[1].shape[0] for e in ev if e[0] == "search")
    assert nq == ts.n_requests
    live = set(live.tolist())
    seen_new = set()
    for e in ev:
        if e[0] == "search":
            assert e[1].dtype == np.float32 and e[1].shape[1] == spec.d
            np.testing.assert_allclose(np.linalg.norm(e[1], axis=1), 1.0, rtol=1e-5)
        elif e[0] == "insert":
            x, ids = e[1], e[2]
            assert x.shape == (ids.size, spec.d)
            assert ids.size == round(0.02 * len(live))
            assert not (set(ids.tolist()) & live) and not (set(ids.tolist()) & seen_new)
            seen_new |= set(ids.tolist())
            live |= set(ids.tolist())
        else:
            ids = e[1]
            assert len(set(ids.tolist())) == ids.size and set(ids.tolist()) <= live
            live -= set(ids.tolist())
    kinds = [e[0] for e in ev]
    assert kinds.count("insert") == kinds.count("delete") == (ts.n_requests - 1) // ts.update_every
    # the trace is a pure function of its seeds
    ev2 = synth.serving_trace(spec, np.arange(spec.n, dtype=np.int64), ts)
    assert all((a[1] == b[1]).all() for a, b in zip(ev, ev2))


def test_trace_skew_and_drift():
    spec = synth.MixtureSpec(key=91, n=1_000, d=8, n_components=40, comp_std=0.01)
    ts = synth.TraceSpec(n_requests=8_000, drift_every=4_000, update_every=10**9, noise_std=0.0)
    ev = synth.serving_trace(spec, np.arange(spec.n, dtype=np.int64), ts)
    assert [e[0] for e in ev] == ["search", "search"]
    means = synth.component_means(spec).astype(np.float32)
    comps = []
    for _, q in ev:
        d2 = ((q[:, None, :] - means[None, :, :]) ** 2).sum(-1)
        comps.append(np.bincount(d2.argmin(1), minlength=spec.n_components))
    for c in comps:
        frac = np.sort(c)[::-1] / c.sum()
        w = (np.arange(40) + 1.0) ** -1.2
        w /= w.sum()
        assert abs(frac[0] - w[0]) < 0.03          # the hottest component takes its Zipf share
    assert comps[0].argmax() != comps[1].argmax()   # the popular set moved


def test_row_labels_follow_location():
    """One label bit per row; a row carries its component's home label
    (component mod 8) with probability 0.7 + 0.3 / 8; masks are one bit,
    uniform over the labels; both are reproducible."""
    spec = synth.MixtureSpec(key=91, n=40_000, d=4, n_components=64, zipf_s=1.1)
    _, comp = synth.database(spec, with_components=True)
    lab = synth.row_labels(spec, comp)
    assert lab.dtype == np.uint32 and (np.bitwise_and(lab, lab - 1) == 0).all() and (lab != 0).all()
    home = (np.uint32(1) << (comp % 8).astype(np.uint32)).astype(np.uint32)
    frac = (lab == home).mean()
    want = 0.7 + 0.3 / 8
    assert abs(frac - want) < 5 * np.sqrt(want * (1 - want) / lab.size)
    assert (synth.row_labels(spec, comp) == lab).all()
    m = synth.query_masks(spec, 16_000)
    assert (np.bitwise_and(m, m - 1) == 0).all()
    counts = np.bincount(np.log2(m).astype(int), minlength=8)
    assert counts.size == 8 and (np.abs(counts - 2000) < 5 * np.sqrt(2000)).all()
