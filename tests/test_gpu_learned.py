"""GPU tests of the learned beam predictor: training kernels against the FP64
oracle, learned search against the oracle's learned search, the exactness of
the learned cut, and what the trained network gains over a fixed beam."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag
from paper_2602_10258_amd import predictor as pred
from workloads import make_config
from workloads.gen import extra_queries

from .parity import tau_for
from .test_gpu_search import gpu_search

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    P[:1024] = rng.normal(0, 0.5, 1024) * scale
    P[1024:1088] = rng.normal(0, 0.1, 64)
    P[1088:5184] = rng.normal(0, 0.2, 4096) * scale
    P[5184:5248] = rng.normal(0, 0.1, 64)
    P[5248:5312] = rng.normal(0, 0.3, 64)
    P[5312] = 2.0
    return P


def test_training_gradient_matches_fp64_oracle():
    import torch
    _say("predictor gradient")
    rng = np.random.default_rng(0)
    for m in (1, 63, 300):
        X = rng.normal(size=(m, 16)).astype(np.float32)
        T = rng.uniform(0, 12, size=m).astype(np.float32)
        P = _params(m)
        loss, g = jag.jag_predictor_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), P)
        lo, go, _ = O.mlp_loss_grad(P.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
        assert abs(loss - lo) <= 1e-4 * max(1.0, abs(lo))
        scale = np.abs(go).max()
        np.testing.assert_allclose(g, go, rtol=1e-4, atol=1e-5 * scale)


def test_training_fits_a_known_function():
    """Minibatch Adam on the GPU drives the loss down on y = 2 x0 - x1 + 3."""
    import torch
    _say("predictor training")
    rng = np.random.default_rng(1)
    X = rng.normal(size=(4096, 16)).astype(np.float32)
    T = (2 * X[:, 0] - X[:, 1] + 3).astype(np.float32)
    P0 = pred.init_params(0)
    P, loss = jag.jag_train_predictor(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), P0,
                                      epochs=30, batch=256, lr=3e-3, seed=2)
    assert np.all(np.isfinite(P))
    assert loss[-1] < 0.02 * loss[0] and loss[-1] < 0.1
    _, _, Y = O.mlp_loss_grad(P.astype(np.float64), X[:64].astype(np.float64), T[:64].astype(np.float64))
    assert np.abs(Y - T[:64]).mean() < 0.3


def _sel_feature(nvalid, n):
    return np.array([np.float32(np.log2(max(v / n, 1e-9)) / 16.0) for v in nvalid], dtype=np.float32)


def test_learned_search_matches_oracle(c1_small):
    """Same BF16 weights on both sides; the oracle evaluates the network in FP64.
    Where the oracle's y + delta is not within 1e-4 of an integer both sides pick
    the same beam, and then the ids must agree (margin rule of tests/parity.py)."""
    w, A, adj, entry = c1_small
    _say("learned search parity")
    P = _params(11, scale=0.3)
    Pq = O.bf16_decode(O.bf16_encode(P))
    ladder = np.array([16, 24, 32, 48, 64, 96, 128], dtype=np.int32)
    rho = 3.0
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=8)
    jag.jag_set_predictor(idx, P, ladder, rho)
    _, _, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 1)
    self_ = _sel_feature(nv, w.n)
    for delta in (-2.0, 0.0, 1.5):
        g = gpu_search(idx, w.Q, w.F, w.pool, 10, 16, learned=1, delta=delta)
        # the first four expansions keep max(128, widest beam) = 128 entries on both sides
        orc = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, 128, 10, learned=Pq, delta=delta,
                       rho=rho, ladder=ladder, sel_feature=self_)
        z = orc.y + delta
        safe = np.abs(z - np.round(z)) > 1e-4
        lh = g["stats"][:, 3]
        assert np.array_equal(lh[safe], orc.lhat[safe]), (delta, lh[safe][:10], orc.lhat[safe][:10])
        same = safe & (orc.margin >= tau_for(0, w.d))
        assert same.mean() >= 0.7
        assert np.array_equal(g["ids"][same], orc.ids[same])
        assert np.array_equal(g["stats"][same, 0], orc.hops[same])
        _say(f"delta={delta} compared {same.sum()} queries exactly; "
             f"beams {np.bincount(lh, minlength=int(ladder[-1]) + 1)[ladder]}")


def test_learned_cut_is_exact(c1_small):
    """With the hop cap out of the way, learned search returns exactly the ids of
    the fixed-beam search at the beam it chose (both on the GPU)."""
    w, A, adj, entry = c1_small
    _say("learned cut exactness")
    ladder = np.array([12, 20, 40, 80, 160], dtype=np.int32)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=8)
    jag.jag_set_predictor(idx, _params(5, scale=0.3), ladder, 1e6)
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, 10, learned=1, delta=0.0)
    lh = g["stats"][:, 3]
    seen = 0
    for L in np.unique(lh):
        sel = lh == L
        f = gpu_search(idx, w.Q[sel], w.F[sel], w.pool, 10, int(L))
        assert np.array_equal(f["ids"], g["ids"][sel]), L
        seen += int(sel.sum())
    assert seen == w.nq


def test_two_pass_schedule_is_exact(c1_small, mixed_world):
    """The default two-pass learned search (run to the prediction and save the
    state, order longest first, resume) returns exactly what one launch in
    submission order returns: ids, distances, counts, expansions and chosen
    beams.  (The distance and attribute counts may differ: the resumed search
    starts its seen-table again from its list, which I1 makes harmless.)"""
    w, A, adj, entry = c1_small
    _say("two-pass learned schedule")
    ladder = np.array([10, 16, 24, 40, 64, 96, 128], dtype=np.int32)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=8)
    cases = [(idx, w.Q, w.F, w.pool, 0)]
    mw, _, madj, mentry = mixed_world
    midx = jag.jag_build_from_graph(mw.X, madj, mentry, scalar=mw.scalar, label_off=mw.loff,
                                    labels=mw.lab, vocab=mw.vocab)
    cases.append((midx, mw.Q, mw.F, mw.pool, 0))
    # a single query; a hop limit below the prediction point (no saved state);
    # a hop limit just past it
    cases.append((idx, w.Q[:1], w.F[:1], w.pool, 0))
    cases.append((idx, w.Q, w.F, w.pool, 3))
    cases.append((midx, mw.Q, mw.F, mw.pool, 6))
    for seed, (ix, Q, F, pool, mh) in enumerate(cases):
        jag.jag_set_predictor(ix, _params(20 + seed, scale=0.4), ladder, 2.5)
        for delta in (-1.0, 0.5, 3.0):
            one = gpu_search(ix, Q, F, pool, 10, 10, learned=1, delta=delta, single_pass=1,
                             max_hops=mh)
            two = gpu_search(ix, Q, F, pool, 10, 10, learned=1, delta=delta, single_pass=0,
                             max_hops=mh)
            for key in ("ids", "d2", "count"):
                assert np.array_equal(one[key], two[key]), (seed, delta, key)
            assert np.array_equal(one["stats"][:, [0, 3]], two["stats"][:, [0, 3]]), (seed, delta)
        _say(f"case {seed}: beams {np.unique(two['stats'][:, 3]).tolist()}")


def test_trace_features_are_beam_independent(c1_small):
    """Trace mode writes the same features for every beam up to 64 (the first four
    expansions keep a 64-entry list), and its answers equal fixed search."""
    w, A, adj, entry = c1_small
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=8)
    a = gpu_search(idx, w.Q, w.F, w.pool, 10, 16, learned=2, features=True)
    b = gpu_search(idx, w.Q, w.F, w.pool, 10, 64, learned=2, features=True)
    f = gpu_search(idx, w.Q, w.F, w.pool, 10, 64)
    assert np.array_equal(a["features"], b["features"])
    assert np.all(a["features"][:, 15] == 1.0)
    onehot = a["features"][:, :4]
    assert np.all(onehot[:, 0] == 1.0) and np.all(onehot[:, 1:] == 0)
    assert np.array_equal(b["ids"], f["ids"])


def test_predictor_gain_mixed_queries():
    """Config-4 shape: c1 vectors with a scalar and 1-3 labels per item, mixed
    label / range / subset queries.  The fitted predictor reaches recall >= 0.95
    on held-out queries with fewer distance computations than the cheapest fixed
    beam that reaches it."""
    import torch
    _say("predictor gain")
    w = make_config("c4", nq=2000)
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=8,
                                     R=32, thresholds=[(0, 1.0), (0, 0.01), (0, 0.0), (1, 0.0)])
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, label_off=w.loff,
                                   labels=w.lab, vocab=8)
    Qt, Ft, pt = extra_queries(w, 20000, qseed=77)
    P, rho, rep = pred.fit(idx, Qt, Ft, pt, k=10)
    _say(f"fit: {rep}")
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10, nthreads=8)

    def run(**kw):
        g = gpu_search(idx, w.Q, w.F, w.pool, 10, kw.pop("L", 10), **kw)
        rec = np.nanmean(O.recall_at_k(g["ids"], gi, gd, nv, 10))
        return rec, g["stats"][:, 1].mean()

    fixed = [(L, *run(L=L)) for L in (10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192)]
    fx = [f for f in fixed if f[1] >= 0.95]
    assert fx, fixed
    cost_fixed = min(f[2] for f in fx)
    learned = [(d, *run(learned=1, delta=d)) for d in (-1.0, -0.5, 0.0, 0.5, 1.0, 2.0, 3.0)]
    lx = [x for x in learned if x[1] >= 0.95]
    _say("fixed", fixed)
    _say("learned", learned)
    assert lx, learned
    cost_learned = min(x[2] for x in lx)
    assert cost_learned < cost_fixed, (cost_learned, cost_fixed)
