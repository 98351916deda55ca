"""GPU parity at the shapes the benchmarks use, beyond the small worlds:

* FP8 E4M3 store at d = 100 (the serving shard's rows: two 16-byte chunks per
  lane) with the FP32 rerank, mixed filter types;
* beams of 512 and 1,024 on the label-set workload's shape (d = 128, 16-wide
  label rows, subset and (a AND b) OR c filters), FP32 and BF16 + rerank;
* the selectivity estimate in the filter records against the oracle's
  estimate (exact counts for label and range filters, label independence
  otherwise);
* the predictor's features at the fourth expansion against the oracle's;
* BF16 and FP8 rows whose lane share is wider than 32 elements (d = 160 and
  150), where the FP32 rescoring switches to its four-lane layout.
Each search is compared twice: with the FP64 oracle under the margin rule
of tests/parity.py, and with the oracle's contract mode (FP32 distances in
the kernel's documented lane order), where every query must return the same
ids and bit-identical distances."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag
from workloads import FILTER_SUBSET, make_config

from .parity import compare, compare_strict, lane_order, tau_for
from .test_gpu_search import _valid_fn, gpu_search

pytestmark = pytest.mark.gpu

LW, S = jag.ATTR_LABELS_WEIGHTED, jag.ATTR_SCALAR


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _index(w, adj, entry, store, keep_f32):
    return jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, label_off=w.loff, labels=w.lab,
                                    vocab=w.vocab, store=store, keep_f32=keep_f32)


@pytest.fixture(scope="module")
def c5_shape():
    """20,000 points of the serving recipe (d = 100, a scalar and 1-5 Zipf
    labels of 1,000, the four filter types), device-built graph with its five
    comparator entries."""
    w = make_config("c5", n=20000, nq=160)
    _say("c5-shape graph", w.X.shape)
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab,
                                     R=48, thresholds=[(S, 1.0), (S, 0.01), (S, 0.0), (LW, 0.01), (LW, 0.0)],
                                     seed=2, device=True)
    return w, O.attrs_of(w), adj, entry


@pytest.mark.parametrize("L,rerank", [(32, 4), (128, 4), (128, 0)])
def test_fp8_two_chunk_rows_match_oracle(c5_shape, L, rerank):
    w, A, adj, entry = c5_shape
    assert w.d == 100
    idx = _index(w, adj, entry, jag.STORE_FP8_E4M3, keep_f32=True)
    _say("fp8 d=100 L", L, "rerank", rerank)
    base = O.fp8_decode_rows(*O.fp8_encode_rows(w.X))
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, L, rerank_mult=rerank)
    orc = O.search(base, adj, entry, A, w.Q, w.F, w.pool, L, 10, rerank=w.X if rerank else None,
                   rerank_mult=rerank or 4, nthreads=8)
    tau = tau_for(jag.STORE_FP8_E4M3, w.d, rerank_d=w.d if rerank else None)
    n_ex, n_fl, n_fd = compare(g["ids"], g["d2"], g["count"], orc, tau, _valid_fn(w, w.F, w.pool),
                               f"fp8 d=100 L={L} rerank={rerank}")
    _say(f"exact {n_ex} flagged {n_fl} flagged-differing {n_fd}; expansions equal "
         f"{np.mean(g['stats'][:, 0] == orc.hops):.3f}")
    # FP8 codes keep 3 mantissa bits, so decoded rows share many coordinates and
    # far more keys sit within the FP32 rounding bound of each other than with
    # FP32 rows (a third of the queries at L = 128); the contract-mode oracle
    # follows the kernel's summation order, so there every query must agree
    assert n_ex >= 0.5 * w.nq
    orc_c = O.search(base, adj, entry, A, w.Q, w.F, w.pool, L, 10, rerank=w.X if rerank else None,
                     rerank_mult=rerank or 4, nthreads=8, contract=lane_order(jag.STORE_FP8_E4M3, w.d))
    compare_strict(g["ids"], g["d2"], g["count"], orc_c, f"fp8 d=100 L={L} rerank={rerank} (contract)")
    assert np.array_equal(g["stats"][:, 0], orc_c.hops)


@pytest.fixture(scope="module")
def c3_shape():
    """20,000 points of the label-set recipe (d = 128, 1-10 Zipf labels of
    1,000: 16-wide label rows), weighted-label graph from the device builder;
    the subset queries with at least one valid item."""
    w = make_config("c3", n=20000, nq=400)
    _say("c3-shape graph", w.X.shape)
    adj, entry = jag.jag_build_graph(w.X, label_off=w.loff, labels=w.lab, vocab=w.vocab, R=64,
                                     thresholds=[(LW, 1.0), (LW, 0.01), (LW, 0.0)], seed=4, device=True)
    A = O.attrs_of(w)
    keep = w.F[:, 0] == FILTER_SUBSET
    _, _, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 1, nthreads=8)
    keep &= nv > 0
    keep[np.flatnonzero(keep)[48:]] = False  # 48 queries: long searches in the oracle
    return w, A, adj, entry, np.flatnonzero(keep)


@pytest.mark.parametrize("L,store", [(512, jag.STORE_F32), (1024, jag.STORE_F32), (512, jag.STORE_BF16)])
def test_long_beams_on_label_set_rows_match_oracle(c3_shape, L, store):
    w, A, adj, entry, sel = c3_shape
    quant = store != jag.STORE_F32
    idx = _index(w, adj, entry, store, keep_f32=quant)
    assert idx.info().label_width == 16
    Q, F = w.Q[sel], w.F[sel]
    _say("c3 shape subset queries", len(sel), "L", L, "store", store)
    g = gpu_search(idx, Q, F, w.pool, 10, L, rerank_mult=4 if quant else 0)
    base = O.bf16_decode(O.bf16_encode(w.X)) if quant else w.X
    orc = O.search(base, adj, entry, A, Q, F, w.pool, L, 10, rerank=w.X if quant else None, rerank_mult=4,
                   nthreads=8)
    tau = tau_for(store, w.d, rerank_d=w.d if quant else None)

    def valid(q, ids):
        return bool(np.all(O.dist_f(A, ids, F, np.full(len(ids), q), w.pool) == 0))

    n_ex, n_fl, n_fd = compare(g["ids"], g["d2"], g["count"], orc, tau, valid, f"L={L} store={store}")
    _say(f"exact {n_ex} flagged {n_fl} flagged-differing {n_fd}; mean expansions {orc.hops.mean():.0f}")
    # over hundreds of expansions some pair of keys nearly always falls within
    # the FP32 rounding bound, so the FP64 margin rule certifies few queries;
    # those it does not must still be valid and ordered (checked above), and
    # against the contract-mode oracle every query must agree exactly
    assert n_fd <= 0.05 * len(sel)
    orc_c = O.search(base, adj, entry, A, Q, F, w.pool, L, 10, rerank=w.X if quant else None, rerank_mult=4,
                     nthreads=8, contract=lane_order(store, w.d))
    compare_strict(g["ids"], g["d2"], g["count"], orc_c, f"L={L} store={store} (contract)")
    assert np.array_equal(g["stats"][:, 0], orc_c.hops)


def test_selectivity_estimate_matches_oracle(mixed_world, c5_shape):
    """The records' estimate (inclusion-exclusion over the clauses) equals the
    oracle's (enumeration of the filter's label assignments)."""
    for w, A, adj, entry in (mixed_world, c5_shape):
        idx = _index(w, adj, entry, jag.STORE_F32, keep_f32=False)
        rec = jag.jag_encode_filters(idx, w.F, w.pool)
        lib_sel = rec[:, 28:32].copy().view(np.float32)[:, 0].astype(np.float64)
        lib_feat = rec[:, 24:28].copy().view(np.float32)[:, 0]
        want = O.selectivity(A, w.F, w.pool)
        np.testing.assert_allclose(lib_sel, want, rtol=2e-7, atol=1e-12)
        np.testing.assert_allclose(lib_feat, O.sel_feature(want), rtol=0, atol=2e-7)
        _say("selectivity", w.name, "types", np.bincount(w.F[:, 0]).tolist(), "ok")


@pytest.mark.parametrize("world", ["c1", "mixed"])
def test_trace_features_match_oracle(c1_small, mixed_world, world):
    """Trace mode's features (the first four expansions on a 64-entry list)
    against the oracle's learned search with a constant network whose beam
    is the ladder's widest, 64 (the same list width)."""
    w, A, adj, entry = c1_small if world == "c1" else mixed_world
    idx = _index(w, adj, entry, jag.STORE_F32, keep_f32=False)
    L = 32
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, L, learned=2, features=True)
    P = np.zeros(O.N_PARAMS, dtype=np.float32)
    P[5312] = 20.0
    sf = O.sel_feature(O.selectivity(A, w.F, w.pool))
    orc = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L, 10, learned=P, ladder=np.array([32, 64], np.int32),
                   sel_feature=sf)
    ok = (orc.margin >= tau_for(0, w.d)) & ~np.isnan(orc.feat[:, 0])
    assert ok.mean() >= 0.7
    gf, of = g["features"][ok].astype(np.float64), orc.feat[ok]
    exact_slots = [0, 1, 2, 3, 9, 10, 11, 12, 13, 14, 15]
    np.testing.assert_allclose(gf[:, exact_slots], of[:, exact_slots], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gf[:, 4], of[:, 4], rtol=0, atol=2e-7)
    np.testing.assert_allclose(gf[:, 5:9], of[:, 5:9], rtol=1e-5, atol=1e-9)
    _say(f"{world}: features of {ok.sum()} queries equal the oracle's")


def test_slot_server_on_the_serving_shape(c5_shape):
    """The resident serving waves at the serving shard's shape (FP8 rows of
    d = 100, two chunks per lane, scalar and label attributes, all four
    filter types, FP32 rerank): every answer equals the direct search's and,
    through it, the contract-mode oracle's."""
    from .test_gpu_serving import _collect
    w, A, adj, entry = c5_shape
    idx = _index(w, adj, entry, jag.STORE_FP8_E4M3, keep_f32=True)
    sp = jag.SearchParams(L=64, rerank_mult=4)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 64, rerank_mult=4)
    base = O.fp8_decode_rows(*O.fp8_encode_rows(w.X))
    orc = O.search(base, adj, entry, A, w.Q, w.F, w.pool, 64, 10, rerank=w.X, rerank_mult=4, nthreads=8,
                   contract=lane_order(jag.STORE_FP8_E4M3, w.d))
    compare_strict(ref["ids"], ref["d2"], ref["count"], orc, "fp8 d=100 L=64 (contract)")
    s = jag.jag_server_start(idx, 10, sp, slot_admission=True)
    try:
        res = _collect(s, jag.jag_server_submit(s, w.Q, w.F, w.pool))
    finally:
        jag.jag_server_stop(s)
    for q, (ids, d, c, lat) in enumerate(res):
        assert c == ref["count"][q] and np.array_equal(ids, ref["ids"][q]), q
        assert np.array_equal(d.view(np.uint32), ref["d2"][q].view(np.uint32)), q
    _say("slot server on the serving shape:", len(res), "answers equal")


@pytest.fixture(scope="module")
def wide_rows():
    """4,000 points of the range recipe with vectors of 150 and 160
    dimensions: BF16 rows of 320 bytes (five chunks per lane) and FP8 rows
    of 154 bytes padded to 192 (three chunks of 16 codes), lane shares wide
    enough that the FP32 rescoring takes its four-lane layout."""
    from workloads.gen import mixture
    w0 = make_config("c2", n=4000, nq=96)
    out = {}
    for d in (150, 160):
        rng = np.random.default_rng(d)
        X, C = mixture(rng, w0.X.shape[0], d, 32)
        Q, _ = mixture(np.random.default_rng(d + 1), w0.Q.shape[0], d, 32, centers=C)
        w = dataclasses.replace(w0, X=X, Q=Q)
        adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, R=32,
                                         thresholds=[(S, 1.0), (S, 0.01), (S, 0.0)], seed=3, device=True)
        out[d] = (w, O.attrs_of(w), adj, entry)
    return out


@pytest.mark.parametrize("store,d", [(jag.STORE_BF16, 160), (jag.STORE_FP8_E4M3, 150)])
def test_wide_rows_rescoring_matches_oracle(wide_rows, store, d):
    w, A, adj, entry = wide_rows[d]
    assert w.d == d
    order = lane_order(store, d)
    assert order[3:5] == [4, 4] and order[1] * order[2] > 32, order  # the four-lane rescoring layout
    _say("wide rows store", store, "d", d)
    idx = _index(w, adj, entry, store, keep_f32=True)
    base = (O.bf16_decode(O.bf16_encode(w.X)) if store == jag.STORE_BF16
            else O.fp8_decode_rows(*O.fp8_encode_rows(w.X)))
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, 48, rerank_mult=4)
    orc = O.search(base, adj, entry, A, w.Q, w.F, w.pool, 48, 10, rerank=w.X, rerank_mult=4, nthreads=8)
    n_ex, n_fl, n_fd = compare(g["ids"], g["d2"], g["count"], orc, tau_for(store, d, rerank_d=d),
                               _valid_fn(w, w.F, w.pool), f"wide rows store={store} d={d}")
    _say(f"exact {n_ex} flagged {n_fl} flagged-differing {n_fd}")
    orc_c = O.search(base, adj, entry, A, w.Q, w.F, w.pool, 48, 10, rerank=w.X, rerank_mult=4, nthreads=8,
                     contract=order)
    compare_strict(g["ids"], g["d2"], g["count"], orc_c, f"wide rows store={store} d={d} (contract)")


def test_learned_fp8_search_matches_oracle(c5_shape):
    """The learned beam over the FP8 store with the FP32 rerank: the same BF16
    network on both sides (the oracle evaluates it in FP64, so queries whose
    y + delta lies within 1e-4 of an integer are left out), distances in the
    kernel's lane order; where both pick the same beam every query returns
    the same ids, distances and count, in one pass and in two."""
    from .test_gpu_learned import _params
    w, A, adj, entry = c5_shape
    P = _params(13, scale=0.3)
    Pq = O.bf16_decode(O.bf16_encode(P))
    ladder = np.array([16, 24, 32, 48, 64, 96, 128], dtype=np.int32)
    rho = 3.0
    idx = _index(w, adj, entry, jag.STORE_FP8_E4M3, keep_f32=True)
    jag.jag_set_predictor(idx, P, ladder, rho)
    base = O.fp8_decode_rows(*O.fp8_encode_rows(w.X))
    sf = O.sel_feature(O.selectivity(A, w.F, w.pool))
    for delta in (0.0, 1.5):
        # the first four expansions keep the widest beam's 128 entries on both sides
        orc = O.search(base, adj, entry, A, w.Q, w.F, w.pool, 128, 10, rerank=w.X, rerank_mult=4,
                       learned=Pq, delta=delta, rho=rho, ladder=ladder, sel_feature=sf, nthreads=8,
                       contract=lane_order(jag.STORE_FP8_E4M3, w.d))
        z = orc.y + delta
        safe = np.abs(z - np.round(z)) > 1e-4
        assert safe.mean() >= 0.9
        for single in (1, 0):
            _say("learned fp8 d=100 delta", delta, "single pass" if single else "two passes")
            g = gpu_search(idx, w.Q, w.F, w.pool, 10, 16, learned=1, delta=delta, rerank_mult=4,
                           single_pass=single)
            lh = g["stats"][:, 3]
            assert np.array_equal(lh[safe], orc.lhat[safe]), (delta, lh[safe][:10], orc.lhat[safe][:10])
            assert np.array_equal(g["ids"][safe], orc.ids[safe])
            assert np.array_equal(g["count"][safe], orc.count[safe])
            for q in np.flatnonzero(safe):
                c = int(g["count"][q])
                assert np.array_equal(g["d2"][q, :c].astype(np.float64), orc.d2[q, :c]), q
            assert np.array_equal(g["stats"][safe, 0], orc.hops[safe])
        _say(f"delta={delta}: {safe.sum()} of {w.nq} queries compared; beams "
             f"{np.bincount(lh, minlength=int(ladder[-1]) + 1)[ladder].tolist()}")
