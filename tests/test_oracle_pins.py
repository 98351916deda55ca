"""Pins for the oracle's graph construction (Algorithm 3), the predictor's
forward pass and features, and the FP32 rerank, each against values the
definitions fix by hand (no second implementation of the same arithmetic).

* Insert + JointRobustPrune: two five-point line worlds built by hand in
  ``tests/golden/build_line_worlds.txt`` (reverse edges, the re-prune of an
  over-full vertex, the alpha test, bucket caps, the union of the expanded
  sets of several threshold searches).  The library's host builder, given the
  same order and thresholds in rounds of one point, must give the same graph.
* Forward pass of the 16-64-64-1 network: torch float64 on random non-zero
  weights (a transposed W1 or W2 changes the output).
* Features at the fourth expansion: a 1-D world whose search is worked by hand.
* Rerank: with rescoring vectors unrelated to the search store, the answer is
  the exact filtered top-k of the rescoring vectors.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import FILTER_BOOLEAN, FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, encode_filters

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "build_line_worlds.txt")


def load_build_cases():
    cases, cur = {}, None
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, *vals = line.split()
        if key == "case":
            cur = cases.setdefault(vals[0], {"points": [], "rows": {}})
        elif key == "points":
            cur["points"].append([float(v) for v in vals])
        elif key == "row":
            cur["rows"][int(vals[0])] = [int(v) for v in vals[1:]]
        elif key == "thresholds":
            cur["thresholds"] = [float(v) for v in vals]
        elif key == "order":
            cur["order"] = np.array([int(v) for v in vals], dtype=np.int32)
        else:
            cur[key] = int(vals[0])
    return cases


CASES = load_build_cases()


def _world(case):
    pts = np.array(case["points"])
    n = len(pts)
    assert np.array_equal(pts[:, 0], np.arange(n))
    X = pts[:, 1:2].astype(np.float32)
    scal = pts[:, 2].astype(np.int32)
    want = np.array([case["rows"][i] for i in range(n)], dtype=np.int32)
    return X, scal, want


def test_golden_build_cases_parse():
    assert sorted(CASES) == ["single_threshold_exhaustive", "two_thresholds_beam_one"]
    for c in CASES.values():
        assert len(c["rows"]) == 5 and all(len(r) == c["R"] for r in c["rows"].values())


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_build_matches_hand_worked_graph(name):
    c = CASES[name]
    X, scal, want = _world(c)
    n = X.shape[0]
    kinds = [O.KIND_SCALAR] * len(c["thresholds"])
    adj, entry, thr = O.build(X, O.Attrs(n, scal, None, None), c["R"], c["lb"], 1.2, kinds,
                              c["thresholds"], seed=0, order=c["order"])
    assert entry == c["order"][0]
    assert np.array_equal(adj, want), f"\n{adj}\n!=\n{want}"


@pytest.mark.parametrize("name", sorted(CASES))
def test_library_host_builder_matches_hand_worked_graph(name):
    from paper_2602_10258_amd import jag
    c = CASES[name]
    X, scal, want = _world(c)
    thr = [(jag.ATTR_SCALAR, q) for q in c["thresholds"]]
    tv = np.array([[np.inf if q >= 1 else 0.0 for q in c["thresholds"]]] * X.shape[0], dtype=np.float32)
    adj, entry = jag.jag_build_graph(X, scalar=scal, R=c["R"], L_build=c["lb"], thresholds=thr, max_batch=1,
                                     order=c["order"], thr_values=tv, n_threads=1)
    assert entry == c["order"][0]
    assert np.array_equal(adj, want), f"\n{adj}\n!=\n{want}"


def test_oracle_build_rejects_a_bad_order():
    c = CASES["single_threshold_exhaustive"]
    X, scal, _ = _world(c)
    with pytest.raises(ValueError):
        O.build(X, O.Attrs(5, scal, None, None), 2, 8, 1.2, [O.KIND_SCALAR], [1.0],
                order=np.array([0, 1, 2, 3, 4], np.int32))  # the entry vertex is 2


def test_oracle_build_given_thresholds_equal_sampled_ones():
    """Handing the sampled thresholds back in reproduces the same graph."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(300, 5)).astype(np.float32)
    scal = rng.integers(0, 1000, size=300).astype(np.int32)
    A = O.Attrs(300, scal, None, None)
    order = np.empty(300, np.int32)
    a1, e1, t1 = O.build(X, A, 8, 16, 1.2, [0, 0, 0], [1.0, 0.05, 0.0], seed=4, order_out=order)
    a2, e2, _ = O.build(X, A, 8, 16, 1.2, [0, 0, 0], [0.5, 0.5, 0.5], seed=99, order=order, thresholds=t1)
    assert e1 == e2 and np.array_equal(a1, a2)


# ---------------------------------------------------------------- network

def _random_net(seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 0.4, size=O.N_PARAMS).astype(np.float32)
    P[1024:1088] = rng.normal(0.2, 0.3, 64)  # biases keep about half the units active
    P[5184:5248] = rng.normal(0.2, 0.3, 64)
    return P


def _torch_forward(P, X):
    P = torch.tensor(P.astype(np.float64))
    x = torch.tensor(X)
    W1, b1 = P[:1024].reshape(64, 16), P[1024:1088]
    W2, b2 = P[1088:5184].reshape(64, 64), P[5184:5248]
    w3, b3 = P[5248:5312], P[5312]
    return (torch.relu(torch.relu(x @ W1.T + b1) @ W2.T + b2) @ w3 + b3).numpy()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mlp_forward_matches_torch_on_nonzero_nets(seed):
    P = _random_net(seed)
    X = np.random.default_rng(seed + 10).normal(size=(128, 16))
    y = O.mlp_forward(P, X)
    want = _torch_forward(P, X)
    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-12)
    assert np.std(want) > 0.1  # the check is not on a near-constant output
    # the loss/gradient routine's forward output (pinned to torch autograd) agrees too
    _, _, Y = O.mlp_loss_grad(P.astype(np.float64), X, np.zeros(len(X)))
    np.testing.assert_allclose(y, Y, rtol=1e-12, atol=1e-12)
    # the check would see a transposed W2
    Pt = P.copy()
    Pt[1088:5184] = P[1088:5184].reshape(64, 64).T.ravel()
    assert np.max(np.abs(O.mlp_forward(Pt, X) - want)) > 1e-3


# ---------------------------------------------------------------- features

def test_learned_features_hand_worked():
    """Ten points on a line, x_i = i = scalar_i, out-edges i -> i+1, i+2, i-1;
    entry 0; query at x = 9 with the range filter [7, 8].  Keys (dist_F, d^2):
    hop 1 expands 0 (7, 81) and finds 1 (6, 64), 2 (5, 49); hop 2 expands
    2 (5, 49): 3 (4, 36), 4 (3, 25); hop 3 expands 4 (3, 25): 5 (2, 16),
    6 (1, 9); hop 4 expands 6 (1, 9): 7 (0, 4), 8 (0, 1).  The list then
    holds 9 entries led by 8 (0, 1), two of them valid.  Features: one-hot
    range, the selectivity feature as given, d^2 of expansions 2-4 over the
    first (49, 25, 9)/81, the best entry's 1/81, squash(x) = x/(1+x) of the
    expanded dist_F 7, 5, 3, 1 and of the best entry's 0, 2/9 valid, 1."""
    n = 10
    X = np.arange(n, dtype=np.float32)[:, None]
    A = O.Attrs(n, np.arange(n, dtype=np.int32), None, None)
    adj = np.full((n, 3), -1, dtype=np.int32)
    for i in range(n):
        nb = [j for j in (i + 1, i + 2, i - 1) if 0 <= j < n]
        adj[i, :len(nb)] = nb
    F, pool = encode_filters([FILTER_RANGE], [(7, 8)])
    Q = np.full((1, 1), 9.0, dtype=np.float32)
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    P[5312] = 10.0  # constant network: the widest ladder beam, no cut
    r = O.search(X, adj, 0, A, Q, F, pool, L=16, k=1, learned=P, sel_feature=np.array([-0.3125], np.float32),
                 ladder=np.array([16, 32], np.int32))
    want = [0, 1, 0, 0, -0.3125, 49 / 81, 25 / 81, 9 / 81, 1 / 81, 7 / 8, 5 / 6, 3 / 4, 1 / 2, 0.0, 2 / 9, 1.0]
    np.testing.assert_allclose(r.feat[0], want, rtol=1e-12, atol=1e-15)
    assert r.ids[0, 0] == 8 and r.lhat[0] == 32


def test_features_absent_without_four_expansions():
    n = 3
    X = np.arange(n, dtype=np.float32)[:, None]
    A = O.Attrs(n, np.arange(n, dtype=np.int32), None, None)
    adj = np.array([[1], [2], [-1]], dtype=np.int32)
    F, pool = encode_filters([FILTER_RANGE], [(0, 2)])
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    r = O.search(X, adj, 0, A, np.zeros((1, 1), np.float32), F, pool, L=16, k=1, learned=P,
                 ladder=np.array([16], np.int32))
    assert np.all(np.isnan(r.feat[0])) and r.hops[0] == 3


# ---------------------------------------------------------------- rerank

def _rerank_world(seed, n=40, d=5):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    X2 = rng.normal(size=(n, d)).astype(np.float32)  # rescoring vectors unrelated to X
    sets = [sorted(rng.choice(4, size=rng.integers(1, 3), replace=False).tolist()) for _ in range(n)]
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    A = O.Attrs(n, rng.integers(0, 50, size=n).astype(np.int32), loff, lab)
    kinds = [FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_BOOLEAN] * 3
    pays = []
    for t in kinds:
        pays.append(int(rng.integers(0, 4)) if t == FILTER_LABEL else (5, 40) if t == FILTER_RANGE
                    else [0, 1] if t == FILTER_SUBSET else [[0], [~1, 2]])
    F, pool = encode_filters(kinds, pays)
    Q = rng.normal(size=(len(kinds), d)).astype(np.float32)
    adj = np.array([[j for j in range(n) if j != i] for i in range(n)], dtype=np.int32)
    return X, X2, A, F, pool, Q, adj


def test_rerank_of_the_whole_list_is_the_exact_answer_on_the_rescoring_vectors():
    """Complete graph, l_s = n: the final list holds every vertex; rescoring all
    4k = n of them and re-sorting gives the exact filtered top-k by the
    rescoring vectors' distances (and, without the re-sort, the store's)."""
    X, X2, A, F, pool, Q, adj = _rerank_world(0)
    n, k = X.shape[0], 10
    r = O.search(X, adj, 0, A, Q, F, pool, L=n, k=k, rerank=X2, rerank_mult=n // k)
    gi, gd, nv = O.bruteforce(X2, A, Q, F, pool, k)
    assert np.array_equal(r.ids, gi)
    np.testing.assert_array_equal(r.d2[gi >= 0], gd[gi >= 0])
    g1, _, _ = O.bruteforce(X, A, Q, F, pool, k)
    assert not np.array_equal(g1, gi)  # the two orders differ, so a missing re-sort would show


def test_rerank_of_a_prefix_resorts_the_store_top_entries():
    """Rescoring only the best m*k = k entries: the answer is the store's exact
    top-k set, ordered by the rescoring vectors."""
    X, X2, A, F, pool, Q, adj = _rerank_world(1)
    n, k = X.shape[0], 6
    r = O.search(X, adj, 0, A, Q, F, pool, L=n, k=k, rerank=X2, rerank_mult=1)
    g1, _, nv = O.bruteforce(X, A, Q, F, pool, k)
    moved = 0
    for q in range(Q.shape[0]):
        ids = [int(v) for v in g1[q] if v >= 0]
        d2 = [float(((X2[v].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum()) for v in ids]
        want = [v for _, v in sorted(zip(d2, ids))]
        assert r.ids[q, :len(want)].tolist() == want
        np.testing.assert_allclose(r.d2[q, :len(want)], sorted(d2), rtol=1e-12)
        moved += want != ids
    assert moved >= Q.shape[0] // 2


# ---------------------------------------------------------------- selectivity

def _labels_world(sets, scal=None):
    n = len(sets)
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    return O.Attrs(n, scal, loff, lab)


def test_selectivity_estimate_hand_worked():
    """Items {0}, {0,1}, {1}, {}: each label held by half of them.  Label 0:
    2/4 (a count); subset {0,1}: 1/2 * 1/2; (0 and 1) or not 0: 1/4 + 1/2 (the
    clauses exclude each other); (0) or (1): 1 - 1/4; range [5, 7] over
    scalars 1, 5, 7, 9: 2/4."""
    A = _labels_world([[0], [0, 1], [1], []], scal=np.array([1, 5, 7, 9], np.int32))
    F, pool = encode_filters([FILTER_LABEL, FILTER_SUBSET, FILTER_BOOLEAN, FILTER_BOOLEAN, FILTER_RANGE],
                             [0, [0, 1], [[0, 1], [~0]], [[0], [1]], (5, 7)])
    np.testing.assert_allclose(O.selectivity(A, F, pool), [0.5, 0.25, 0.75, 0.75, 0.5], rtol=1e-15)


def test_selectivity_estimate_against_exact_counts_under_independent_labels():
    """Labels drawn independently per item: the estimate is the probability a
    random item passes, so the exact count (Pre-Filtering) must lie within a
    few binomial standard deviations of n times the estimate; label and range
    estimates are the exact fraction."""
    rng = np.random.default_rng(12)
    n = 100_000
    p = np.array([0.5, 0.4, 0.3, 0.2, 0.1, 0.05, 0.6, 0.7])
    held = rng.random((n, len(p))) < p
    sets = [np.flatnonzero(r).tolist() for r in held]
    scal = rng.integers(0, 1000, size=n).astype(np.int32)
    A = _labels_world(sets, scal)
    kinds = [FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_SUBSET, FILTER_BOOLEAN, FILTER_BOOLEAN,
             FILTER_BOOLEAN, FILTER_SUBSET]
    pays = [3, (100, 349), [0, 1], [0, 1, 2, 6], [[0, 1], [2]], [[0, ~1], [3]], [[~0], [1, 2], [5, ~6]],
            [4, 5]]
    F, pool = encode_filters(kinds, pays)
    est = O.selectivity(A, F, pool)
    X = np.zeros((n, 1), np.float32)
    _, _, nv = O.bruteforce(X, A, np.zeros((len(kinds), 1), np.float32), F, pool, 1)
    frac = nv / n
    np.testing.assert_allclose(est[:2], frac[:2], rtol=1e-12)
    sd = np.sqrt(est * (1 - est) / n)
    assert np.all(np.abs(est - frac) <= 6 * sd + 1e-12), (est, frac)
    # the estimate follows the true independent probabilities too
    true = [p[0] * p[1], p[0] * p[1] * p[2] * p[6], p[0] * p[1] + p[2] - p[0] * p[1] * p[2],
            p[0] * (1 - p[1]) + p[3] - p[0] * (1 - p[1]) * p[3]]
    np.testing.assert_allclose(est[[2, 3, 4, 5]], true, rtol=0.05)


def test_selectivity_estimate_assumes_independence():
    """With label 1 held only together with label 0 the subset {0, 1} passes
    whatever holds label 1, but the estimate multiplies the two frequencies."""
    A = _labels_world([[0, 1], [0], [0], [2]])
    F, pool = encode_filters([FILTER_SUBSET], [[0, 1]])
    assert O.selectivity(A, F, pool)[0] == pytest.approx(0.75 * 0.25)


# ---------------------------------------------------------------- contract order

def test_contract_mode_search_agrees_with_fp64():
    """The FP32 lane-order distances stay within the rounding bound of the FP64
    ones: on a world of small integer coordinates every sum is exact, so the
    two modes return the same ids and distances; on Gaussian data every query
    whose FP64 margin clears the bound returns the same ids."""
    from tests.parity import lane_order, tau_for
    X, A, Q, F, pool, *_ = _tiny_world_for_contract()
    n = X.shape[0]
    adj = np.array([[(i + j) % n for j in range(1, 9)] for i in range(n)], dtype=np.int32)
    Xi = np.round(X * 4).astype(np.float32)
    Qi = np.round(Q * 4).astype(np.float32)
    for store in (0, 1, 2):
        con = lane_order(store, X.shape[1])
        a = O.search(Xi, adj, 0, A, Qi, F, pool, 24, 10, rerank=Xi, rerank_mult=2, contract=con)
        b = O.search(Xi, adj, 0, A, Qi, F, pool, 24, 10, rerank=Xi, rerank_mult=2)
        assert np.array_equal(a.ids, b.ids) and np.array_equal(a.d2, b.d2)
        c = O.search(X, adj, 0, A, Q, F, pool, 24, 10, contract=con)
        e = O.search(X, adj, 0, A, Q, F, pool, 24, 10)
        ok = e.margin >= tau_for(store, X.shape[1])
        assert ok.mean() > 0.5 and np.array_equal(c.ids[ok], e.ids[ok])
        np.testing.assert_allclose(c.d2[c.ids >= 0], e.d2[e.ids >= 0], rtol=1e-5)


def _tiny_world_for_contract(seed=6, n=300, d=37):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    sets = [sorted(rng.choice(5, size=rng.integers(1, 3), replace=False).tolist()) for _ in range(n)]
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    A = O.Attrs(n, rng.integers(0, 100, size=n).astype(np.int32), loff, lab)
    kinds = [FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_BOOLEAN] * 6
    pays = [int(rng.integers(0, 5)) if t == FILTER_LABEL else (10, 80) if t == FILTER_RANGE
            else [0, 2] if t == FILTER_SUBSET else [[1], [3, ~4]] for t in kinds]
    F, pool = encode_filters(kinds, pays)
    Q = rng.normal(size=(len(kinds), d)).astype(np.float32)
    return X, A, Q, F, pool
