"""Parity at the headline workload's full size (range filters, 1M x 96,
R = 64, 10,000 queries in one launch, as the benchmark launches them): the
GPU answers every query; the oracle answers a sample of 250 on the same graph
(Algorithms 1 and 2; the beam predictor with the same BF16 weights), and the
sampled outputs must agree under the margin rule of tests/parity.py."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag
from workloads import make_config

from .parity import compare, tau_for
from .test_gpu_search import _valid_fn, gpu_search

pytestmark = pytest.mark.gpu

S = jag.ATTR_SCALAR
LADDER = np.array([10, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 56, 64], dtype=np.int32)


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c2_full():
    w = make_config("c2")
    _say("c2 full size: building the graph on the device")
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, R=w.R, L_build=2 * w.R, seed=0, device=True,
                                     thresholds=[(S, 1.0), (S, 0.01), (S, 0.0)])
    qs = np.arange(0, w.nq, w.nq // 250)
    return w, O.attrs_of(w), adj, entry, qs


def _check(w, A, orc, g, qs, tau, what):
    n_ex, n_fl, n_fd = compare(g["ids"][qs], g["d2"][qs], g["count"][qs], orc, tau,
                               _valid_fn(w, w.F[qs], w.pool), what)
    _say(f"{what}: exact {n_ex} flagged {n_fl} flagged-differing {n_fd}")
    assert n_ex >= 0.9 * len(qs)
    return n_ex


def test_fullsize_fp32_fixed_beam(c2_full):
    w, A, adj, entry, qs = c2_full
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar)
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, 44)
    orc = O.search(w.X, adj, entry, A, w.Q[qs], w.F[qs], w.pool, 44, 10, nthreads=16)
    _check(w, A, orc, g, qs, tau_for(0, w.d), "c2 full fp32 L=44")
    same = orc.margin >= tau_for(0, w.d)
    assert np.array_equal(g["stats"][qs][same, 0], orc.hops[same])
    gi, gd, nv = O.bruteforce(w.X, A, w.Q[qs], w.F[qs], w.pool, 10, nthreads=16)
    rec = float(np.nanmean(O.recall_at_k(g["ids"][qs], gi, gd, nv, 10)))
    _say(f"recall@10 of the sample {rec:.4f}")
    assert rec >= 0.9


def test_fullsize_bf16_rerank_fixed_beam(c2_full):
    w, A, adj, entry, qs = c2_full
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, store=jag.STORE_BF16, keep_f32=True)
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, 44, rerank_mult=4)
    base = O.bf16_decode(O.bf16_encode(w.X))
    orc = O.search(base, adj, entry, A, w.Q[qs], w.F[qs], w.pool, 44, 10, rerank=w.X, rerank_mult=4,
                   nthreads=16)
    _check(w, A, orc, g, qs, tau_for(1, w.d, rerank_d=w.d), "c2 full bf16+rerank L=44")


@pytest.mark.parametrize("delta", [0.0, 2.0])
def test_fullsize_learned_two_pass(c2_full, delta):
    """The benchmark's operating mode: learned beam (two passes), BF16 store,
    FP32 rerank of the best 40; random BF16 weights on both sides."""
    w, A, adj, entry, qs = c2_full
    rng = np.random.default_rng(5)
    P = (rng.normal(size=5313) * 0.3).astype(np.float32)
    Pq = O.bf16_decode(O.bf16_encode(P))
    rho = 3.0
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, store=jag.STORE_BF16, keep_f32=True)
    jag.jag_set_predictor(idx, P, LADDER, rho)
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, 16, learned=1, delta=delta, rerank_mult=4)
    s = np.sort(w.scalar)
    cnt = np.searchsorted(s, w.F[qs, 3], side="right") - np.searchsorted(s, w.F[qs, 2], side="left")
    sel = np.array([np.float32(np.log2(max(c / w.n, 1e-9)) / 16.0) for c in cnt], dtype=np.float32)
    base = O.bf16_decode(O.bf16_encode(w.X))
    orc = O.search(base, adj, entry, A, w.Q[qs], w.F[qs], w.pool, int(LADDER[-1]), 10, rerank=w.X,
                   rerank_mult=4, learned=Pq, delta=delta, rho=rho, ladder=LADDER, sel_feature=sel, nthreads=16)
    z = orc.y + delta
    safe = np.abs(z - np.round(z)) > 1e-4
    lh = g["stats"][qs, 3]
    assert np.array_equal(lh[safe], orc.lhat[safe])
    tau = tau_for(1, w.d, rerank_d=w.d)
    same = safe & (orc.margin >= tau)
    _say(f"learned delta={delta}: beams {np.bincount(lh, minlength=65)[LADDER]}, compared {same.sum()} exactly")
    assert same.mean() >= 0.8
    assert np.array_equal(g["ids"][qs][same], orc.ids[same])
    assert np.array_equal(g["stats"][qs][same, 0], orc.hops[same])
