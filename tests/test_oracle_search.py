"""Pins for the oracle's search (Algorithms 1-2), prune (Algorithm 4), build
(Algorithm 3, structural invariants only) and exact filtered k-NN."""
import collections

import numpy as np
import pytest

from oracle import oracle as O
from workloads import (FILTER_BOOLEAN, FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, encode_filters,
                       make_config)


def _tiny_world(seed=0, n=160, d=6):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    sets = [sorted(rng.choice(6, size=rng.integers(1, 4), replace=False).tolist()) for _ in range(n)]
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    scal = rng.integers(0, 100, size=n).astype(np.int32)
    A = O.Attrs(n, scal, loff, lab)
    kinds, pays = [], []
    for i in range(24):
        t = i % 4
        if t == FILTER_LABEL:
            pays.append(int(rng.integers(0, 6)))
        elif t == FILTER_RANGE:
            lo = int(rng.integers(0, 90))
            pays.append((lo, lo + int(rng.integers(0, 30))))
        elif t == FILTER_SUBSET:
            pays.append(sorted(rng.choice(6, size=2, replace=False).tolist()))
        else:
            a, b, c = rng.choice(6, size=3, replace=False).tolist()
            pays.append([[a, b], [~c]])
        kinds.append(t)
    F, pool = encode_filters(kinds, pays)
    Q = rng.normal(size=(len(kinds), d)).astype(np.float32)
    return X, A, Q, F, pool, sets, scal, kinds, pays


def _ring_random_graph(n, R, seed):
    """Strongly connected: edge i -> i+1 (mod n) plus random out-edges."""
    rng = np.random.default_rng(seed)
    adj = np.full((n, R), -1, dtype=np.int32)
    for i in range(n):
        nb = [(i + 1) % n]
        for v in rng.permutation(n):
            if len(nb) >= R - 1:
                break
            if v != i and v not in nb and rng.random() < 0.5:
                nb.append(int(v))
        adj[i, :len(nb)] = nb
    return adj


def test_exhaustive_beam_equals_bruteforce():
    """With l_s >= n nothing is ever evicted, so every reachable vertex is expanded
    and Query returns exactly the filtered top-k (Algorithm 1 semantics)."""
    X, A, Q, F, pool, *_ = _tiny_world()
    n = X.shape[0]
    adj = _ring_random_graph(n, 8, 1)
    res = O.search(X, adj, 0, A, Q, F, pool, L=n, k=10)
    gi, gd, nv = O.bruteforce(X, A, Q, F, pool, 10)
    assert np.array_equal(res.ids, gi)
    assert np.array_equal(res.count, np.minimum(nv, 10))
    np.testing.assert_array_equal(res.d2[gi >= 0], gd[gi >= 0])
    assert np.all(res.hops == n)  # every vertex expanded


@pytest.mark.parametrize("L", [10, 16, 40])
def test_complete_graph_gives_exact_answer(L):
    """On a complete graph the entry's expansion discovers every vertex, so the
    beam is the global top-l_s by D_F and the answer is the exact filtered top-k."""
    X, A, Q, F, pool, *_ = _tiny_world(seed=2, n=60)
    n = X.shape[0]
    adj = np.array([[j for j in range(n) if j != i] for i in range(n)], dtype=np.int32)
    res = O.search(X, adj, 5, A, Q, F, pool, L=L, k=10)
    gi, gd, nv = O.bruteforce(X, A, Q, F, pool, 10)
    assert np.array_equal(res.ids, gi)


def test_bruteforce_matches_set_semantics():
    """Exact filtered k-NN: valid items are those with g = 1 (Section 2), ranked by
    (distance, id); the number of distance computations is the number of valid items."""
    X, A, Q, F, pool, sets, scal, kinds, pays = _tiny_world(seed=4)
    gi, gd, nv = O.bruteforce(X, A, Q, F, pool, 10)
    for q in range(len(kinds)):
        t, p = kinds[q], pays[q]
        valid = []
        for i in range(X.shape[0]):
            s = set(sets[i])
            ok = (p in s) if t == FILTER_LABEL else (p[0] <= scal[i] <= p[1]) if t == FILTER_RANGE \
                else (set(p) <= s) if t == FILTER_SUBSET \
                else any(all((l in s) if l >= 0 else ((~l) not in s) for l in cl) for cl in p)
            if ok:
                valid.append(i)
        assert nv[q] == len(valid)
        d = ((X[valid].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.array(valid), d))[:10]
        want = np.full(10, -1)
        want[:len(order)] = np.array(valid)[order]
        assert np.array_equal(gi[q], want)


def test_figure2_style_range_walk():
    """A 1-D line of points whose attribute equals their position.  From x=0 the
    range filter [3,5] pulls the search along the path towards the range even with
    a beam of one: dist_F decreases at every step and the walk stops at the valid
    item nearest the query (the Figure 2 example's behaviour)."""
    n = 10
    X = np.arange(n, dtype=np.float32)[:, None]
    A = O.Attrs(n, np.arange(n, dtype=np.int32), None, None)
    adj = np.full((n, 2), -1, dtype=np.int32)
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n]
        adj[i, :len(nb)] = nb
    F, pool = encode_filters([FILTER_RANGE], [(3, 5)])
    Q = np.zeros((1, 1), dtype=np.float32)
    res = O.search(X, adj, 0, A, Q, F, pool, L=1, k=1)
    assert res.ids[0, 0] == 3 and res.count[0] == 1
    assert res.hops[0] == 4  # expands 0, 1, 2, 3
    res3 = O.search(X, adj, 0, A, Q, F, pool, L=8, k=3)
    assert res3.ids[0].tolist() == [3, 4, 5]


def test_results_are_valid_sorted_distinct(c1_small):
    w, A, adj, entry = c1_small
    res = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=32, k=10)
    for q in range(w.nq):
        ids = res.ids[q, :res.count[q]]
        assert len(set(ids.tolist())) == len(ids)
        assert np.all(w.lab[ids] == w.F[q, 1])  # single-label items: equality
        assert np.all(np.diff(res.d2[q, :res.count[q]]) >= 0)


def test_recall_grows_with_beam(c1_small):
    w, A, adj, entry = c1_small
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10)
    rec = []
    for L in (16, 64, 256):
        r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=L, k=10)
        rec.append(np.nanmean(O.recall_at_k(r.ids, gi, gd, nv, 10)))
    assert rec[0] <= rec[1] <= rec[2]
    assert rec[1] >= 0.95 and rec[2] >= 0.99


def test_constant_predictor_equals_fixed_beam(c1_small):
    """A predictor whose output is the constant c picks Lhat = ladder[ceil(c + delta)];
    running the first four expansions untruncated and then cutting to Lhat must give
    exactly the fixed-Lhat search (the learned mode's exactness argument)."""
    w, A, adj, entry = c1_small
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    for c, delta, want in ((1.0, 0.0, 24), (3.4, 0.0, 64), (3.4, 1.0, 96), (0.2, -5.0, 16)):
        P[5312] = c
        r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=512, k=10, learned=P, delta=delta)
        assert np.all(r.lhat == want)
        f = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=want, k=10)
        assert np.array_equal(r.ids, f.ids)


def test_hop_cap_stops_search(c1_small):
    w, A, adj, entry = c1_small
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    P[5312] = 4.0  # Lhat = 64
    r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=512, k=10, learned=P, rho=0.25)
    assert np.all(r.hops <= 16)


def test_rerank_with_same_vectors_is_identity(c1_small):
    w, A, adj, entry = c1_small
    a = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=64, k=10)
    b = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L=64, k=10, rerank=w.X, rerank_mult=4)
    assert np.array_equal(a.ids, b.ids)


# ---------------------------------------------------------------- prune

def _prune_case(points, attrs, R, quant_kinds_thr, p=0, cand=None):
    X = np.asarray(points, dtype=np.float32)
    n = X.shape[0]
    A = O.Attrs(n, np.asarray(attrs, dtype=np.int32), None, None)
    kinds = [O.KIND_SCALAR] * len(quant_kinds_thr)
    thr = np.tile(np.asarray(quant_kinds_thr, dtype=np.float64), (n, 1))
    cand = list(range(1, n)) if cand is None else cand
    return O.prune(X, A, R, 1.2, kinds, thr, p, cand)


def test_prune_alpha_rule_collinear():
    """Points at 1, 2, 3 on a ray from p: 1.2*dist(1,2)=1.2 < 2 and 1.2*dist(1,3)=2.4 < 3,
    so 1 dominates both; points on opposite sides are both kept."""
    assert _prune_case([[0], [1], [2], [3]], [0, 0, 0, 0], 8, [np.inf]) == [1]
    assert _prune_case([[0], [1], [-1.1]], [0, 0, 0], 8, [np.inf]) == [1, 2]


def test_prune_alpha_rule_is_strict():
    """Keep v only if alpha*dist(u,v) > dist(p,v): equality prunes (Algorithm 4)."""
    # u at 5, v at 6 -> alpha*dist(u,v) = 1.2*1 = 1.2 < 6; v at -0.6 (d=0.6), u at 0.5:
    # dist(u,v) = 1.1 -> 1.32 > 0.6 keep.  Exact tie: u at 1, v at 6: 1.2*5 = 6 = dist(p,v).
    assert _prune_case([[0], [1], [6]], [0, 0, 0], 8, [np.inf]) == [1]
    assert _prune_case([[0], [1], [-6]], [0, 0, 0], 8, [np.inf]) == [1, 2]


def test_prune_bucket_cap():
    """Six well-separated directions, R=4, one threshold: the bucket closes at
    ceil(0.9*4/1) = 4 vertices, taken in distance order."""
    ang = np.arange(6) * np.pi / 3
    rad = 1.0 + 0.01 * np.arange(6)
    pts = [[0.0, 0.0]] + [[r * np.cos(a), r * np.sin(a)] for a, r in zip(ang, rad)]
    assert _prune_case(pts, [0] * 7, 4, [np.inf]) == [1, 2, 3, 4]
    # R=8 and two thresholds: ceil(0.9*8/2) = 4 per bucket
    assert len(_prune_case(pts, [0] * 7, 8, [np.inf, np.inf])) == 4


def test_prune_earlier_bucket_member_joins_without_test():
    """Appendix D.3: a vertex chosen by an earlier threshold joins the current bucket
    without the alpha test, counts towards its cap and so can close it early.
    Geometry (p at the origin, R=4, T={inf, 0} -> cap 2 per bucket):
      a=(-1,0) attr 9, v1=(1.9,0.3) attr 1, v2=(2,0) attr 0, w=(0,2.5) attr 2.
    Bucket t=inf (vector order a, v1, v2, w) keeps {a, v1} and closes.
    Bucket t=0 (attribute order v2, v1, w, a) takes v2, then v1 (already chosen,
    no test) and closes, so w is never added: result [a, v1, v2].  Testing v1
    against v2 would have rejected it and let w in."""
    pts = [[0, 0], [-1, 0], [1.9, 0.3], [2, 0], [0, 2.5]]
    attrs = [0, 9, 1, 0, 2]
    assert _prune_case(pts, attrs, 4, [np.inf, 0.0]) == [1, 2, 3]


def test_prune_threshold_zero_orders_by_attribute_first():
    """t = 0: candidates are visited strictly by attribute distance (Section 4
    ablation: 0% = compare by filter distance first)."""
    pts = [[0], [1], [10], [-10]]
    attrs = [0, 50, 1, 2]
    # attribute order 2 (|1|), 3 (|2|), 1 (|50|); 2 and 3 lie on opposite sides,
    # 1 is dominated by neither (1.2*9 > 1 and 1.2*11 > 1)
    assert _prune_case(pts, attrs, 8, [0.0]) == [2, 3, 1]


# ---------------------------------------------------------------- build

def _reachable(adj, s):
    seen = {s}
    dq = collections.deque([s])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if v >= 0 and v not in seen:
                seen.add(int(v))
                dq.append(int(v))
    return seen


def test_build_invariants(c1_small):
    """Build is parity unpinned (no reference graph): check its structure."""
    w, A, adj, entry = c1_small
    n, R = adj.shape
    assert R == 32
    deg = (adj >= 0).sum(1)
    assert deg.max() <= R and deg.min() >= 1
    for i in range(0, n, 97):
        row = adj[i][adj[i] >= 0]
        assert i not in row.tolist()
        assert len(set(row.tolist())) == len(row)
        assert np.all(adj[i][deg[i]:] == -1)  # padding only at the end
    # pruning can drop every in-edge of a vertex; the paper does not repair that
    assert len(_reachable(adj, entry)) >= 0.999 * n
    # entry = point nearest the centroid
    cen = w.X.astype(np.float64).mean(0)
    assert entry == int(np.argmin(((w.X.astype(np.float64) - cen) ** 2).sum(1)))


def test_build_deterministic_and_quantile_thresholds():
    w = make_config("c4", n=600, nq=4)
    A = O.attrs_of(w)
    kinds = [O.KIND_SCALAR, O.KIND_SCALAR, O.KIND_SCALAR, O.KIND_LABELS]
    quant = [1.0, 0.01, 0.0, 0.5]
    a1, e1, t1 = O.build(w.X, A, 16, 32, 1.2, kinds, quant, seed=3)
    a2, e2, t2 = O.build(w.X, A, 16, 32, 1.2, kinds, quant, seed=3)
    assert e1 == e2 and np.array_equal(a1, a2)
    assert np.all(np.isinf(t1[:, 0])) and np.all(t1[:, 2] == 0)
    # 1% of 500 samples = 5th smallest |a_p - a_v|: about 1% of the range domain
    assert 0 < np.median(t1[:, 1]) < 0.03 * 1_000_000
    deg = (a1 >= 0).sum(1)
    assert deg.max() <= 16
    assert len(_reachable(a1, e1)) >= 0.99 * 600


def test_weight_entries_reach_the_threshold_limits():
    """Weight-JAG entries (comparator w * dist_A + dist, Section 3.4) at their
    two limits give exactly the Threshold-JAG graphs: w = 0 orders by vector
    distance alone (threshold 100 %), a weight far above every vector distance
    orders by attribute first (threshold 0)."""
    rng = np.random.default_rng(12)
    n = 500
    X = rng.normal(0, 1, size=(n, 8)).astype(np.float32)
    scal = rng.integers(0, 60, size=n).astype(np.int32)
    sets = [sorted(rng.choice(12, size=rng.integers(1, 4), replace=False).tolist()) for _ in range(n)]
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    A = O.Attrs(n, scal, loff, lab)
    W = O.WEIGHT_ENTRY
    for kind in (O.KIND_SCALAR, O.KIND_LABELS):
        g0, e0, t0 = O.build(X, A, 12, 24, 1.2, [kind | W], [0.0], seed=4)
        gi, ei, _ = O.build(X, A, 12, 24, 1.2, [kind], [1.0], seed=4)
        assert e0 == ei and np.array_equal(g0, gi), kind
        assert np.all(t0 == 0)
        gw, ew, tw = O.build(X, A, 12, 24, 1.2, [kind | W], [1e6], seed=4)
        gz, ez, _ = O.build(X, A, 12, 24, 1.2, [kind], [0.0], seed=4)
        assert ew == ez and np.array_equal(gw, gz), kind
        # the weight is the multiplier times sigma / sigma_A > 0
        assert np.all(tw > 0)
    # a middle weight gives a graph of its own, valid and searchable
    gm, em, _ = O.build(X, A, 12, 24, 1.2, [O.KIND_SCALAR, O.KIND_SCALAR | W], [1.0, 2.0], seed=4)
    assert (gm >= 0).sum(1).max() <= 12
    assert len(_reachable(gm, em)) >= 0.99 * n
