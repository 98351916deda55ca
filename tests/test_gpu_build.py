"""GPU graph construction (Algorithms 3 and 4 with the App. D.3 notes;
Section 3.4 for weight entries) against the oracle and the host builder.

* Rounds of one point with the oracle's insertion order and thresholds: the
  device builder performs the oracle's sequential construction, so the graphs
  agree edge for edge.
* Default rounds: the device builder forms every value in the host builder's
  order (canonical FP32 distance, one fused multiply-add per weight entry),
  so it gives the host builder's graph edge for edge, for every comparator
  kind, odd and large dimensions included."""
import sys

import numpy as np
import pytest

from paper_2602_10258_amd import jag
from workloads import make_config

from .test_build_parity import CASES, WEIGHTED_CASES, oracle_graph, small_world, weighted_oracle_graph

pytestmark = pytest.mark.gpu

W = jag.THRESHOLD_WEIGHT
S, LB, LW = jag.ATTR_SCALAR, jag.ATTR_LABELS, jag.ATTR_LABELS_WEIGHTED


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", ["scalar", "labels", "mixed5", "weight", "deg128"])
def test_device_rounds_of_one_give_the_oracle_graph(case):
    n, d, R, lb, thr = CASES[case]
    X, scal, loff, lab = small_world(n, d, seed=len(case))
    oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, R, lb, thr, seed=3)
    _say("device build, rounds of one:", case, n, d, R)
    adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=12, R=R, L_build=lb,
                                     thresholds=thr, max_batch=1, order=order, thr_values=tv, device=True)
    assert entry == oentry
    assert np.array_equal(adj, oadj), f"{np.sum(np.any(adj != oadj, axis=1))} rows differ"


@pytest.mark.parametrize("case", sorted(WEIGHTED_CASES))
def test_device_weighted_labels_rounds_of_one_give_the_oracle_graph(case):
    """App. D.3's frequency-weighted label distance, with thresholds halfway
    between consecutive distinct distances (see test_build_parity)."""
    X, scal, loff, lab, R, lb, thr, tv, order, oadj, oentry = weighted_oracle_graph(case)
    _say("device build, rounds of one, weighted labels:", case, X.shape, R)
    adj, entry = jag.jag_build_graph(X, scalar=scal, label_off=loff, labels=lab, vocab=24, R=R, L_build=lb,
                                     thresholds=thr, max_batch=1, order=order, thr_values=tv, device=True)
    assert entry == oentry
    assert np.array_equal(adj, oadj), f"{np.sum(np.any(adj != oadj, axis=1))} rows differ"


def _world(name):
    if name == "c1":
        w = make_config("c1")
        return w, dict(label_off=w.loff, labels=w.lab, vocab=w.vocab), 32, [(LB, 1.0), (LB, 0.0)]
    if name == "c2":
        w = make_config("c2", n=20000, nq=10)
        return w, dict(scalar=w.scalar), 64, [(S, 1.0), (S, 0.01), (S, 0.0)]
    if name == "c2r128":
        w = make_config("c2", n=20000, nq=10)
        return w, dict(scalar=w.scalar), 128, [(S, 1.0), (S, 0.01), (S, 0.0)]
    if name == "c2w":
        w = make_config("c2", n=20000, nq=10)
        return w, dict(scalar=w.scalar), 48, [(S | W, 0.0), (S | W, 10.0), (S | W, 1000.0)]
    if name == "c3":
        w = make_config("c3", n=20000, nq=10)
        return w, dict(label_off=w.loff, labels=w.lab, vocab=w.vocab), 32, [(LW, 1.0), (LW, 0.01), (LW, 0.0)]
    if name == "c5":
        w = make_config("c5", n=20000, nq=10)
        return (w, dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab), 40,
                [(S, 1.0), (S, 0.01), (S, 0.0), (LW, 0.01), (LB, 0.0)])
    raise KeyError(name)


@pytest.mark.parametrize("name", ["c1", "c2", "c2w", "c3", "c5", "c2r128"])
def test_device_build_equals_host_build(name):
    w, attrs, R, thr = _world(name)
    kw = dict(R=R, thresholds=thr, seed=11, **attrs)
    _say("host build", name, w.X.shape, R, thr)
    hadj, hentry = jag.jag_build_graph(w.X, **kw)
    _say("device build", name)
    dadj, dentry = jag.jag_build_graph(w.X, device=True, **kw)
    assert dentry == hentry
    diff = np.sum(np.any(dadj != hadj, axis=1))
    _say("rows differing", diff, "mean degree", float(np.mean(np.sum(dadj >= 0, axis=1))))
    assert diff == 0


@pytest.mark.parametrize("d", [37, 200])
def test_device_build_odd_and_large_dimensions(d):
    X, scal, loff, lab = small_world(3000, d, seed=d)
    kw = dict(scalar=scal, label_off=loff, labels=lab, vocab=12, R=24,
              thresholds=[(S, 1.0), (LB, 0.0), (S | W, 5.0)], seed=2)
    hadj, he = jag.jag_build_graph(X, **kw)
    _say("device build d =", d)
    dadj, de = jag.jag_build_graph(X, device=True, **kw)
    assert de == he and np.array_equal(dadj, hadj)


def test_device_build_index_and_limits():
    X, scal, loff, lab = small_world(500, 16, seed=9)
    with pytest.raises(jag.JagError):  # the device beam holds at most 256
        jag.jag_build_graph(X, scalar=scal, R=16, L_build=300, thresholds=[(S, 1.0)], device=True)
    _say("jag_build on the device")
    idx = jag.jag_build(X, scalar=scal, R=16, thresholds=[(S, 1.0), (S, 0.0)], device=True, seed=4)
    hadj, he = jag.jag_build_graph(X, scalar=scal, R=16, thresholds=[(S, 1.0), (S, 0.0)], seed=4)
    adj, e = jag.jag_get_graph(idx)
    assert e == he and np.array_equal(adj, hadj)


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_device_tiny_worlds_match_the_oracle(n):
    from .test_build_parity import S as S_
    X, scal, loff, lab = small_world(n, 4, seed=n)
    thr = [(S_, 1.0), (S_, 0.0)]
    oadj, oentry, tv, order = oracle_graph(X, scal, loff, lab, 4, 8, thr, seed=1)
    _say("device build, tiny world n =", n)
    adj, entry = jag.jag_build_graph(X, scalar=scal, R=4, L_build=8, thresholds=thr, max_batch=1,
                                     order=order, thr_values=tv, device=True)
    assert entry == oentry and np.array_equal(adj, oadj)


def test_device_duplicates_small_beams_and_eight_entries_match_the_oracle():
    rng = np.random.default_rng(4)
    X = np.repeat(rng.normal(size=(40, 8)).astype(np.float32), 5, axis=0)
    scal = np.repeat(rng.integers(0, 4, size=40), 5).astype(np.int32)
    loff = np.arange(X.shape[0] + 1, dtype=np.int64)
    lab = np.zeros(X.shape[0], np.int32)
    cases = [(X, scal, loff, lab, 1, 8, 16, [(S, 1.0), (S, 0.0), (LB, 0.0)])]
    X2, s2, lo2, la2 = small_world(300, 12, seed=8)
    cases += [(X2, s2, lo2, la2, 12, R, lb, thr) for R, lb, thr in
              [(1, 1, [(S, 1.0)]), (6, 1, [(S, 1.0), (S, 0.0)]),
               (16, 20, [(S, 1.0), (S, 0.5), (S, 0.2), (S, 0.05), (S, 0.0), (LB, 1.0), (LB, 0.0), (S | W, 3.0)])]]
    for X_, s_, lo_, la_, voc, R, lb, thr in cases:
        oadj, oentry, tv, order = oracle_graph(X_, s_, lo_, la_, R, lb, thr, seed=5)
        _say("device build, rounds of one:", X_.shape, R, lb, len(thr))
        adj, entry = jag.jag_build_graph(X_, scalar=s_, label_off=lo_, labels=la_, vocab=voc, R=R, L_build=lb,
                                         thresholds=thr, max_batch=1, order=order, thr_values=tv, device=True)
        assert entry == oentry and np.array_equal(adj, oadj), (X_.shape, R, lb, len(thr))


@pytest.mark.parametrize("d", [1, 512])
def test_device_build_smallest_and_largest_dimension(d):
    X, scal, loff, lab = small_world(2000, d, seed=d)
    kw = dict(scalar=scal, R=16, thresholds=[(S, 1.0), (S, 0.01), (S, 0.0)], seed=3)
    hadj, he = jag.jag_build_graph(X, **kw)
    _say("device build d =", d)
    dadj, de = jag.jag_build_graph(X, device=True, **kw)
    assert de == he and np.array_equal(dadj, hadj)


def test_device_build_hub_vertices_take_the_global_memory_prune():
    """Identical points all link to the same vertex: a round of 8,192 of them
    gives it more in-links than one LDS prune holds, so its prune runs with
    its arrays in global memory; the graph still equals the host builder's."""
    X = np.zeros((20000, 8), np.float32)
    scal = np.zeros(20000, np.int32)
    kw = dict(scalar=scal, R=8, thresholds=[(S, 1.0), (S, 0.0)], max_batch=20000)
    _say("device build of 20,000 identical points, rounds up to 8,192")
    dadj, de = jag.jag_build_graph(X, device=True, **kw)
    hadj, he = jag.jag_build_graph(X, **kw)
    assert de == he and np.array_equal(dadj, hadj)
    # and the same at a degree above 64 with mixed rows
    X2, s2, lo2, la2 = small_world(6000, 16, seed=3)
    X2[:3000] = X2[0]
    kw2 = dict(scalar=s2, R=96, thresholds=[(S, 1.0), (S, 0.0)], max_batch=6000)
    dadj, de = jag.jag_build_graph(X2, device=True, **kw2)
    hadj, he = jag.jag_build_graph(X2, **kw2)
    assert de == he and np.array_equal(dadj, hadj)


@pytest.mark.parametrize("cap", ["64", "256"])
def test_device_build_global_memory_prunes_for_insertions_and_reverse_edges(monkeypatch, cap):
    """With the LDS capacity of a prune lowered (JAG_BUILD_LDS_CANDIDATES),
    insertion prunes and reverse-edge prunes go through the global-memory
    pass (all of them at 64, some at 256); the graph is still the host's."""
    w = make_config("c2", n=20000, nq=10)
    kw = dict(scalar=w.scalar, R=64, thresholds=[(S, 1.0), (S, 0.01), (S, 0.0)], seed=5)
    hadj, he = jag.jag_build_graph(w.X, **kw)
    monkeypatch.setenv("JAG_BUILD_LDS_CANDIDATES", cap)
    _say("device build with prunes of more than", cap, "candidates in global memory")
    dadj, de = jag.jag_build_graph(w.X, device=True, **kw)
    assert de == he and np.array_equal(dadj, hadj)
