"""GPU tests of general Boolean filters given as truth tables (Section 2's
arbitrary Boolean predicate; dist_F of Section 3.1 = fewest flips to a true
assignment): search and Pre-Filtering against the oracle, and the encoding
rules for the variable-size distance tables."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag
from workloads import FILTER_RANGE, FILTER_TABLE, Workload, encode_filters, make_config

from .parity import compare, tau_for
from .test_gpu_search import _valid_fn, gpu_search

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _bool_world(nvar, n=4000, nq=96, seed=3):
    """Items hold a random assignment of nvar binary variables (labels
    0..nvar-1); queries are random functions with pass rates from 2^-nvar
    (one true assignment) up to about one half."""
    rng = np.random.default_rng(seed)
    w0 = make_config("c1", n=n, nq=nq)
    bits = rng.random((n, nvar)) < 0.5
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum(bits.sum(1))
    lab = np.nonzero(bits)[1].astype(np.int32)
    kinds, pays = [], []
    N = 1 << nvar
    for i in range(nq):
        m = max(1, int(round(N * 2.0 ** -rng.uniform(1, nvar))))
        tab = np.zeros(N, dtype=bool)
        tab[rng.choice(N, size=m, replace=False)] = True
        vars_ = rng.permutation(nvar).tolist()  # any order of the variables
        kinds.append(FILTER_TABLE)
        pays.append((vars_, tab))
    F, pool = encode_filters(kinds, pays)
    w = Workload(f"bool{nvar}", w0.X, w0.Q, F, pool, None, loff, lab, nvar, k=10, R=32, L=64)
    adj, entry = jag.jag_build_graph(w.X, label_off=loff, labels=lab, vocab=nvar, R=32,
                                     thresholds=[(jag.ATTR_LABELS, 1.0), (jag.ATTR_LABELS, 0.01),
                                                 (jag.ATTR_LABELS, 0.0)], seed=seed)
    return w, O.attrs_of(w), adj, entry


@pytest.mark.parametrize("nvar,L", [(10, 16), (10, 96), (15, 48)])
def test_table_filters_match_oracle(nvar, L):
    nq = 96 if nvar <= 10 else 24   # the oracle evaluates 2^nvar assignments per distance
    w, A, adj, entry = _bool_world(nvar, nq=nq)
    _say("table filters nvar", nvar, "L", L)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    g = gpu_search(idx, w.Q, w.F, w.pool, 10, L)
    orc = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, L, 10, nthreads=8)
    n_ex, n_fl, n_fd = compare(g["ids"], g["d2"], g["count"], orc, tau_for(0, w.d),
                               _valid_fn(w, w.F, w.pool), f"table nvar={nvar} L={L}")
    _say(f"exact {n_ex} flagged {n_fl} flagged-differing {n_fd}")
    assert n_ex >= 0.8 * w.nq
    same = orc.margin >= tau_for(0, w.d)
    assert np.array_equal(g["stats"][same, 0], orc.hops[same])


def test_table_filters_exact_knn():
    import torch
    w, A, adj, entry = _bool_world(10, nq=64, seed=5)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    rec = torch.from_numpy(jag.jag_encode_filters(idx, w.F, w.pool)).cuda()
    Qd = torch.from_numpy(w.Q).cuda()
    k = 10
    ids = torch.empty((w.nq, k), dtype=torch.int32, device="cuda")
    dd = torch.empty((w.nq, k), dtype=torch.float32, device="cuda")
    cnt = torch.empty((w.nq,), dtype=torch.int32, device="cuda")
    jag.jag_exact_knn(idx, Qd, rec, k, ids, dd, cnt)
    torch.cuda.synchronize()
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, k + 1)
    assert np.array_equal(cnt.cpu().numpy(), np.minimum(nv, k))
    ids = ids.cpu().numpy()
    tau = tau_for(0, w.d)
    checked = 0
    for q in range(w.nq):
        gaps = np.diff(gd[q]) / np.maximum(gd[q, 1:], 1e-30)
        if np.all(gaps[np.isfinite(gaps)] >= tau):  # no near-ties among the top k + 1
            assert np.array_equal(ids[q], gi[q, :k]), q
            checked += 1
    assert checked >= 0.8 * w.nq


def test_table_encoding_rules(mixed_world):
    """Tables need the sized encoder; sizes are 2^nvar bytes, 16-byte aligned,
    after the records; records of other types are unchanged by the tables;
    malformed tables and short buffers are rejected."""
    w, A, adj, entry = mixed_world
    idx = jag.jag_build_from_graph(w.X, adj, entry, scalar=w.scalar, label_off=w.loff, labels=w.lab,
                                   vocab=w.vocab)
    tab3 = np.zeros(8, dtype=bool)
    tab3[[1, 6]] = True
    tab6 = np.zeros(64, dtype=bool)
    tab6[5] = True
    F, pool = encode_filters([FILTER_RANGE, FILTER_TABLE, FILTER_TABLE], [(10, 500), ([4, 7, 2], tab3),
                                                                         (list(range(6)), tab6)])
    L = jag.lib()
    import ctypes as C
    need = C.c_int64()
    Fc = np.ascontiguousarray(F, np.int32)
    Pc = np.ascontiguousarray(pool, np.int32)
    jag._check(L.jag_encoded_bytes(idx.handle, jag._ptr(Fc), 3, jag._ptr(Pc), Pc.size, C.byref(need)))
    assert need.value == 3 * 128 + 16 + 64
    buf = jag.jag_encode_filters(idx, F, pool)
    assert buf.size == need.value
    # the range record equals its encoding alone
    assert np.array_equal(buf[:128], jag.jag_encode_filters(idx, F[:1], pool)[0])
    # the non-sized encoder refuses tables; a short buffer is refused
    out = np.zeros((3, 128), dtype=np.uint8)
    assert L.jag_encode_filters(idx.handle, jag._ptr(Fc), 3, jag._ptr(Pc), Pc.size, jag._ptr(out)) == jag.JAG_EINVAL
    short = np.zeros(need.value - 1, dtype=np.uint8)
    assert L.jag_encode_filters_sized(idx.handle, jag._ptr(Fc), 3, jag._ptr(Pc), Pc.size, jag._ptr(short),
                                      short.size) == jag.JAG_EINVAL
    # repeated variable, too many variables, wrong length
    for bad in ([4, 4, 2], list(range(16))):
        tb = np.zeros(1 << len(bad), dtype=bool)
        tb[0] = True
        Fb, pb = encode_filters([FILTER_TABLE], [(bad, tb)])
        with pytest.raises(jag.JagError):
            jag.jag_encode_filters(idx, Fb, pb)
    Fb, pb = encode_filters([FILTER_TABLE], [([1, 2], np.array([True, False, False, True]))])
    Fb[0, 5] += 1
    pb = np.concatenate([pb, [0]]).astype(np.int32)
    with pytest.raises(jag.JagError):
        jag.jag_encode_filters(idx, Fb, pb)
