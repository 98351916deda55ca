"""The no-allocation search entry point against jag_search_encoded: the same
kernels, with the launch order and the two-pass saved states in the
library's fixed device array instead of stream-ordered allocations.  Two
calls in a row per mode, the second with a smaller batch (the array keeps
the first call's contents)."""
import sys

import numpy as np
import pytest

from paper_2602_10258_amd import jag
from workloads import make_config

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _run(fn, idx, Q, rec, k, sp):
    import torch
    nq = Q.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int32, device="cuda")
    d2 = torch.full((nq, k), -1.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((nq,), -7, dtype=torch.int32, device="cuda")
    st = torch.zeros((nq, 4), dtype=torch.int32, device="cuda")
    sp = jag.SearchParams(**{**sp.__dict__, "stats": st})
    fn(idx, Q, rec, k, sp, ids, d2, cnt)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d2.cpu().numpy(), cnt.cpu().numpy(), st.cpu().numpy()


@pytest.fixture(scope="module")
def world():
    import torch
    w = make_config("c2", n=20000, nq=6000)
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, R=32, seed=1, device=True,
                                     thresholds=[(jag.ATTR_SCALAR, 1.0), (jag.ATTR_SCALAR, 0.01),
                                                 (jag.ATTR_SCALAR, 0.0)])
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, store=jag.STORE_BF16, keep_f32=True)
    rng = np.random.default_rng(3)
    P = (rng.normal(0, 0.3, 5313)).astype(np.float32)
    P[5312] = 2.0
    jag.jag_set_predictor(idx, P, np.array([10, 16, 24, 40, 64], np.int32), 2.5)
    Q = torch.from_numpy(w.Q).cuda()
    rec = torch.from_numpy(jag.jag_encode_filters(idx, w.F, w.pool)).cuda()
    return idx, Q, rec


@pytest.mark.parametrize("mode", ["fixed_ordered", "learned_two_pass", "learned_one_pass"])
def test_noalloc_equals_allocating_search(world, mode):
    idx, Q, rec = world
    sp = {"fixed_ordered": jag.SearchParams(L=40, rerank_mult=4),
          "learned_two_pass": jag.SearchParams(L=10, learned=1, delta=0.5, rerank_mult=4),
          "learned_one_pass": jag.SearchParams(L=10, learned=1, delta=0.5, rerank_mult=4, single_pass=1)}[mode]
    for nq in (6000, 4500):  # the second call is smaller (still an ordered batch)
        _say("no-alloc", mode, nq)
        a = _run(jag.jag_search_encoded_noalloc, idx, Q[:nq], rec[:nq], 10, sp)
        b = _run(jag.jag_search_encoded, idx, Q[:nq], rec[:nq], 10, sp)
        for x, y, name in zip(a, b, ("ids", "dists", "count", "stats")):
            if name == "stats" and mode == "learned_two_pass":
                x, y = x[:, [0, 3]], y[:, [0, 3]]  # distance counts depend on the resumed seen-table
            assert np.array_equal(x, y), (mode, nq, name)
        assert np.all(a[2] >= 0) and np.mean(a[2] == 10) > 0.5  # real answers, not untouched buffers


def test_noalloc_rejects_a_batch_beyond_its_scratch(world):
    import torch
    idx, Q, rec = world
    nq = 4_194_305  # one query past the 32 MiB launch-order limit
    big_q = torch.zeros((nq, Q.shape[1]), dtype=torch.float32, device="cuda")
    big_r = rec[:1].repeat(nq, 1)
    ids = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
    d2 = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
    cnt = torch.empty((nq,), dtype=torch.int32, device="cuda")
    with pytest.raises(jag.JagError) as e:
        jag.jag_search_encoded_noalloc(idx, big_q, big_r, 10, jag.SearchParams(L=40), ids, d2, cnt)
    assert e.value.status == jag.JAG_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
