"""The library's graph builder against the oracle's (Algorithms 3 and 4 with
the App. D.3 notes; Section 3.4 for weight entries).

In rounds of one point, with the oracle's insertion order and per-point
thresholds handed in, the library's builder performs exactly the oracle's
sequential construction, so the two graphs must agree edge for edge (the
library in FP32, the oracle in FP64: the small worlds here have no ties
closer than FP32 rounding).  The frequency-weighted label distance (App.
D.3) forms its constant C and its shared-label sums in FP32 in the library
and in FP64 in the oracle; a sampled quantile threshold equals one of the
distances exactly, so rounding could move that distance to either side of
it.  Its parity cases hand both builders thresholds halfway between two
consecutive distinct distances of each point instead, which no rounding of
the sums can cross."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag

W = jag.THRESHOLD_WEIGHT
S, LB = jag.ATTR_SCALAR, jag.ATTR_LABELS
LW = jag.ATTR_LABELS_WEIGHTED

CASES = {
    "scalar": (400, 16, 12, 24, [(S, 1.0), (S, 0.05), (S, 0.0)]),
    "labels": (400, 16, 12, 24, [(LB, 1.0), (LB, 0.1), (LB, 0.0)]),
    "mixed5": (1000, 33, 10, 20, [(S, 1.0), (LB, 0.1), (S, 0.0), (LB, 0.0), (S, 0.2)]),
    "weight": (400, 16, 12, 24, [(S | W, 0.0), (S | W, 2.0), (S | W, 50.0)]),
    "wide": (1500, 40, 20, 40, [(S, 1.0), (S, 0.01), (S, 0.0)]),
    "deg128": (1200, 16, 128, 160, [(S, 1.0), (LB, 0.0)]),
}


def small_world(n, d, seed, vocab=12):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    scal = rng.integers(0, 10**6, size=n).astype(np.int32)
    nl = rng.integers(1, 5, size=n)
    loff = np.zeros(n + 1, np.int64)
    loff[1:] = np.cumsum(nl)
    lab = np.concatenate([np.sort(rng.choice(vocab, size=k, replace=False)) for k in nl]).astype(np.int32)
    return X, scal, loff, lab


def oracle_graph(X, scal, loff, lab, R, lb, thr, seed):
    n = X.shape[0]
    A = O.Attrs(n, scal, loff, lab)
    order = np.empty(n, np.int32)
    adj, entry, tv = O.build(X, A, R, lb, 1.2, [k for k, _ in thr], [q for _, q in thr], seed=seed,
                             order_out=order)
    return adj, entry, tv.astype(np.float32), order


@pytest.mark.parametrize("case", sorted(CASES))
def test_sequential_rounds_give_the_oracle_graph(case):
    n, d, R, lb, thr = CASES[case]
    X, scal, loff, lab = small_world(n, d, seed=len(case))
    oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, R, lb, thr, seed=3)
    assert order[0] == oentry
    adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=12, R=R, L_build=lb,
                                     thresholds=thr, max_batch=1, order=order, thr_values=tv, n_threads=4)
    assert entry == oentry
    assert np.array_equal(adj, oadj), f"{np.sum(np.any(adj != oadj, axis=1))} rows differ"


def test_given_order_and_thresholds_are_checked():
    X, scal, loff, lab = small_world(50, 8, seed=1)
    thr = [(S, 1.0), (S | W, 1.0)]
    kw = dict(scalar=scal, R=8, thresholds=thr, n_threads=2)
    bad_order = np.arange(50, dtype=np.int32)
    bad_order[3] = 4
    with pytest.raises(jag.JagError):
        jag.jag_build_graph(X, order=bad_order, **kw)
    tv = np.zeros((50, 2), np.float32)
    tv[:, 0] = np.inf
    adj, entry = jag.jag_build_graph(X, order=np.arange(50, dtype=np.int32)[::-1].copy(), thr_values=tv, **kw)
    assert entry == 49
    for bad in (np.nan, -1.0):
        tb = tv.copy()
        tb[7, 0] = bad
        with pytest.raises(jag.JagError):
            jag.jag_build_graph(X, thr_values=tb, **kw)
    tb = tv.copy()
    tb[7, 1] = np.inf  # a weight must be finite
    with pytest.raises(jag.JagError):
        jag.jag_build_graph(X, thr_values=tb, **kw)
    with pytest.raises(ValueError):
        jag.jag_build_graph(X, thr_values=tv[:10], **kw)


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_tiny_worlds_match_the_oracle(n):
    X, scal, loff, lab = small_world(n, 4, seed=n)
    thr = [(S, 1.0), (S, 0.0)]
    oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, 4, 8, thr, seed=1)
    adj, entry = jag.jag_build_graph(X, scalar=scal, R=4, L_build=8, thresholds=thr, max_batch=1,
                                     order=order, thr_values=tv, n_threads=2)
    assert entry == oentry and np.array_equal(adj, oadj)


def test_duplicate_vectors_and_equal_attributes_match_the_oracle():
    """Ties in both components fall to the id in both builders."""
    rng = np.random.default_rng(4)
    base = rng.normal(size=(40, 8)).astype(np.float32)
    X = np.repeat(base, 5, axis=0)                      # every vector five times
    scal = np.repeat(rng.integers(0, 4, size=40), 5).astype(np.int32)
    loff = np.arange(X.shape[0] + 1, dtype=np.int64)
    lab = np.zeros(X.shape[0], np.int32)
    thr = [(S, 1.0), (S, 0.0), (LB, 0.0)]
    oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, 8, 16, thr, seed=2)
    adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=1, R=8, L_build=16,
                                     thresholds=thr, max_batch=1, order=order, thr_values=tv, n_threads=2)
    assert entry == oentry and np.array_equal(adj, oadj)


def test_degree_one_beam_one_and_eight_entries_match_the_oracle():
    X, scal, loff, lab = small_world(300, 12, seed=8)
    for R, lb, thr in [(1, 1, [(S, 1.0)]), (6, 1, [(S, 1.0), (S, 0.0)]),
                       (16, 20, [(S, 1.0), (S, 0.5), (S, 0.2), (S, 0.05), (S, 0.0), (LB, 1.0), (LB, 0.0),
                                 (S | W, 3.0)])]:
        oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, R, lb, thr, seed=5)
        adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=12, R=R, L_build=lb,
                                         thresholds=thr, max_batch=1, order=order, thr_values=tv, n_threads=2)
        assert entry == oentry and np.array_equal(adj, oadj), (R, lb, len(thr))


def zipf_label_world(n, d, seed, vocab=24, max_labels=4):
    """Label sets drawn with Zipf-like label frequencies, so that the label
    weights log(1/p_l) are far apart."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    p = 1.0 / np.arange(1, vocab + 1) ** 1.1
    p /= p.sum()
    nl = rng.integers(1, max_labels + 1, size=n)
    sets = [np.sort(rng.choice(vocab, size=k, replace=False, p=p)) for k in nl]
    loff = np.zeros(n + 1, np.int64)
    loff[1:] = np.cumsum(nl)
    lab = np.concatenate(sets).astype(np.int32)
    scal = rng.integers(0, 10**6, size=n).astype(np.int32)
    return X, scal, loff, lab


def midpoint_thresholds(X, scal, loff, lab, thr, seed):
    """Per-point thresholds for the weighted parity cases: each sampled
    quantile threshold (a distance value of the point) is moved halfway to
    the point's next larger distinct distance, then rounded to FP32 (both
    builders get the same FP32 value).  Returns (float32 [n][|T|], order)."""
    n = X.shape[0]
    A = O.Attrs(n, scal, loff, lab)
    order = np.empty(n, np.int32)
    _, _, tv = O.build(X, A, 4, 8, 1.2, [k for k, _ in thr], [q for _, q in thr], seed=seed,
                       order_out=order)
    out = tv.copy()
    for ti, (kind, q) in enumerate(thr):
        if q >= 1.0 or q <= 0.0 or kind & jag.THRESHOLD_WEIGHT:
            continue
        for p in range(n):
            da = O.dist_a(A, kind, np.full(n, p), np.arange(n))
            da = np.delete(da, p)
            t = tv[p, ti]
            above = np.unique(da[da > t * (1 + 1e-9) + 1e-12])
            nxt = above[0] if len(above) else t + 1.0
            assert nxt - t > 1e-4 * max(1.0, abs(t)), (p, t, nxt)  # far from FP32 rounding
            out[p, ti] = (t + nxt) / 2
    return out.astype(np.float32), order


WEIGHTED_CASES = {
    "wlabels": (400, 16, 12, 24, [(LW, 1.0), (LW, 0.1), (LW, 0.0)]),
    "wlabels_mixed": (500, 20, 15, 30, [(S, 1.0), (S, 0.01), (S, 0.0), (LW, 0.05), (LW, 0.0)]),
}


def weighted_oracle_graph(case):
    n, d, R, lb, thr = WEIGHTED_CASES[case]
    X, scal, loff, lab = zipf_label_world(n, d, seed=len(case))
    tv, order = midpoint_thresholds(X, scal, loff, lab, thr, seed=3)
    adj, entry, _ = O.build(X, O.Attrs(n, scal, loff, lab), R, lb, 1.2, [k for k, _ in thr],
                            [q for _, q in thr], order=order, thresholds=tv.astype(np.float64))
    return X, scal, loff, lab, R, lb, thr, tv, order, adj, entry


@pytest.mark.parametrize("case", sorted(WEIGHTED_CASES))
def test_weighted_labels_rounds_of_one_give_the_oracle_graph(case):
    X, scal, loff, lab, R, lb, thr, tv, order, oadj, oentry = weighted_oracle_graph(case)
    adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=24, R=R, L_build=lb,
                                     thresholds=thr, max_batch=1, order=order, thr_values=tv, n_threads=4)
    assert entry == oentry
    assert np.array_equal(adj, oadj), f"{np.sum(np.any(adj != oadj, axis=1))} rows differ"
    assert np.mean(np.sum(oadj >= 0, axis=1)) > R / 2  # a real graph, not an empty one
