"""The library's graph builder against the oracle's (Algorithms 3 and 4 with
the App. D.3 notes; Section 3.4 for weight entries).

In rounds of one point, with the oracle's insertion order and per-point
thresholds handed in, the library's builder performs exactly the oracle's
sequential construction, so the two graphs must agree edge for edge (the
library in FP32, the oracle in FP64: the small worlds here have no ties
closer than FP32 rounding).  The frequency-weighted label distance is left
out: its constant C is an FP32 sum in the library and an FP64 sum in the
oracle, which moves every capped distance by a rounding-sized amount."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag

W = jag.THRESHOLD_WEIGHT
S, LB = jag.ATTR_SCALAR, jag.ATTR_LABELS

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
