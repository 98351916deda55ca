"""Launch order of large batches: a fixed-beam or one-pass learned launch of at
least 4096 queries runs the searches expected to be long first (a device
counting sort over selectivity classes: range filters broadest first, the
label-based ones narrowest first).  No answer may depend on that order: one
launch of 4,640 or 11,200 queries must return, query for query, what
launches of fewer than 4096 queries (submission order) return."""
import sys

import numpy as np
import pytest

from paper_2602_10258_amd import jag

from .test_gpu_learned import _params
from .test_gpu_search import gpu_search

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _tiled(mw, copies=29, seed=3):
    """The mixed world's 160 queries (all four filter types), each repeated
    with a little seeded noise on the vector: 4,640 queries."""
    rng = np.random.default_rng(seed)
    Q = np.concatenate([mw.Q + rng.normal(0, 0.02, size=mw.Q.shape).astype(np.float32)
                        for _ in range(copies)]).astype(np.float32)
    F = np.concatenate([mw.F] * copies)
    return Q, F


def _chunked(ix, Q, F, pool, chunk=2000, **kw):
    parts = [gpu_search(ix, Q[i:i + chunk], F[i:i + chunk], pool, 10, **kw) for i in range(0, len(Q), chunk)]
    return {key: np.concatenate([p[key] for p in parts]) for key in ("ids", "d2", "count", "stats")}


@pytest.mark.parametrize("mode,copies", [("fixed", 29), ("learned_one_pass", 29), ("learned_two_pass", 29),
                                         ("fixed", 70), ("learned_two_pass", 70)])
def test_large_launch_matches_small_launches(mixed_world, mode, copies):
    """copies = 70: 11,200 queries, more than the sort keeps in registers
    (10,240), so its second pass reads the classes again."""
    mw, _, adj, entry = mixed_world
    Q, F = _tiled(mw, copies=copies)
    assert len(Q) >= 4096
    ix = jag.jag_build_from_graph(mw.X, adj, entry, scalar=mw.scalar, label_off=mw.loff, labels=mw.lab,
                                  vocab=mw.vocab)
    if mode == "fixed":
        kw = dict(L=24)
    else:
        jag.jag_set_predictor(ix, _params(41, scale=0.4), np.array([10, 16, 24, 40, 64], dtype=np.int32), 2.5)
        kw = dict(L=10, learned=1, delta=0.5, single_pass=int(mode == "learned_one_pass"))
    _say(f"{mode}: one launch of {len(Q)} queries against launches of 2000")
    big = gpu_search(ix, Q, F, mw.pool, 10, **kw)
    small = _chunked(ix, Q, F, mw.pool, **kw)
    assert np.all(big["count"] >= 0)  # every query written
    for key in ("ids", "d2", "count"):
        assert np.array_equal(big[key], small[key]), key
    cols = [0, 1, 2, 3] if mode != "learned_two_pass" else [0, 3]
    assert np.array_equal(big["stats"][:, cols], small["stats"][:, cols])
