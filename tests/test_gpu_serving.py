"""GPU tests of the request server: results identical alone and in the mix,
admission limits, queue and memory budgets, concurrent submitters."""
import sys
import threading
import time

import numpy as np
import pytest

from paper_2602_10258_amd import jag
from workloads import FILTER_LABEL, encode_filters

from .test_gpu_search import _index, gpu_search

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _collect(s, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            t = int(t)
            if t in out:
                continue
            r = jag.jag_server_poll(s, t)
            if r is not None:
                out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.0005)
    return [out[int(t)] for t in tickets]


def _rows(F, pool, i):
    """Filter row i with its own pool slice (so single requests can be submitted)."""
    f = F[i:i + 1].copy()
    if f[0, 0] in (2, 3):
        p = pool[f[0, 4]:f[0, 4] + f[0, 5]].copy()
        f[0, 4] = 0
        return f, p
    return f, np.zeros(1, np.int32)


@pytest.mark.parametrize("store", [jag.STORE_F32, jag.STORE_BF16])
def test_results_same_alone_and_in_mix(mixed_world, store):
    w, A, adj, entry = mixed_world
    _say("server alone vs mix, store", store)
    idx = _index(w, adj, entry, store=store, keep_f32=True)
    sp = jag.SearchParams(L=48, rerank_mult=4 if store else 0)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 48, rerank_mult=4 if store else 0)
    s = jag.jag_server_start(idx, 10, sp, max_batch=16, n_streams=3, max_wait_us=50)
    try:
        # the mix: everything at once, split into interleaved submissions
        t_mix = np.concatenate([jag.jag_server_submit(s, w.Q[i::4], w.F[i::4], w.pool) for i in range(4)])
        order = np.concatenate([np.arange(i, w.nq, 4) for i in range(4)])
        mix = _collect(s, t_mix)
        # alone: one request at a time, waiting for each
        alone = []
        for i in range(0, w.nq, 7):
            f, p = _rows(w.F, w.pool, i)
            t = jag.jag_server_submit(s, w.Q[i:i + 1], f, p)
            alone.append((i, _collect(s, t)[0]))
        st = jag.jag_server_stats_get(s)
    finally:
        jag.jag_server_stop(s)
    for (ids, d, c, lat), q in zip(mix, order):
        assert np.array_equal(ids, ref["ids"][q]) and c == ref["count"][q]
        assert np.array_equal(d.view(np.uint32), ref["d2"][q].view(np.uint32))
    for i, (ids, d, c, lat) in alone:
        assert np.array_equal(ids, ref["ids"][i]) and c == ref["count"][i]
    assert st["completed"] == w.nq + len(alone)
    assert st["p99_us"] >= st["p50_us"] > 0
    _say(st)


def test_admission_limit_and_overlap(mixed_world):
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=64), max_batch=8, n_streams=4,
                             max_inflight=16, max_wait_us=0)
    try:
        t = jag.jag_server_submit(s, np.repeat(w.Q, 4, 0), np.repeat(w.F, 4, 0), w.pool)
        jag.jag_server_drain(s)
        res = _collect(s, t)
        st = jag.jag_server_stats_get(s)
    finally:
        jag.jag_server_stop(s)
    assert st["max_inflight_seen"] <= 16
    assert st["max_inflight_seen"] > 8  # two batches were on the GPU together
    assert st["completed"] == 4 * w.nq and st["resident_capacity"] > 0
    a = np.stack([r[0] for r in res])
    assert np.array_equal(a[0::4], a[1::4]) and np.array_equal(a[0::4], a[3::4])


def test_queue_budget_and_errors(mixed_world):
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    with pytest.raises(jag.JagError) as e:
        jag.jag_server_start(idx, 10, jag.SearchParams(L=32), max_batch=4096, hbm_budget_bytes=1000)
    assert e.value.status == jag.JAG_EUNSUPPORTED
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=32), max_batch=4, n_streams=1,
                             queue_capacity=10, max_inflight=4)
    try:
        Fbad, pbad = encode_filters([FILTER_LABEL], [999])
        with pytest.raises(jag.JagError) as e:
            jag.jag_server_submit(s, w.Q[:1], Fbad, pbad)
        assert e.value.status == jag.JAG_EINVAL
        with pytest.raises(jag.JagError) as e:
            jag.jag_server_submit(s, w.Q[:11], w.F[:11], w.pool)
        assert e.value.status == jag.JAG_EBUSY
        t = jag.jag_server_submit(s, w.Q[:10], w.F[:10], w.pool)
        jag.jag_server_drain(s)
        assert len(_collect(s, t)) == 10
        with pytest.raises(jag.JagError):
            jag.jag_server_poll(s, 10 ** 9)
    finally:
        jag.jag_server_stop(s)


def test_concurrent_submitters(mixed_world):
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 40)
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=40), max_batch=32, n_streams=4,
                             max_wait_us=100)
    got = {}

    def client(j):
        for i in range(j, w.nq, 4):
            f, p = _rows(w.F, w.pool, i)
            t = jag.jag_server_submit(s, w.Q[i:i + 1], f, p)
            got[i] = t[0]

    try:
        th = [threading.Thread(target=client, args=(j,)) for j in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        res = _collect(s, [got[i] for i in range(w.nq)])
    finally:
        jag.jag_server_stop(s)
    for i, (ids, d, c, lat) in enumerate(res):
        assert np.array_equal(ids, ref["ids"][i])


def test_table_filters_through_the_server():
    """Truth-table filters travel with their distance tables: the server's
    answers equal a direct search, mixed with other filter types, in batches
    that hold several tables and alone."""
    from .test_gpu_table_filters import _bool_world
    w, A, adj, entry = _bool_world(10, nq=64, seed=7)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    # every other query becomes a plain label filter
    from workloads import FILTER_TABLE
    kinds, pays = [], []
    for i in range(w.nq):
        if i % 2:
            kinds.append(FILTER_LABEL)
            pays.append(i % w.vocab)
        else:
            f = w.F[i]
            p = w.pool[f[4]:f[4] + f[5]]
            nv = int(p[0])
            words = p[1 + nv:].astype(np.uint32)
            tab = np.unpackbits(words.view(np.uint8), bitorder="little")[: 1 << nv].astype(bool)
            kinds.append(FILTER_TABLE)
            pays.append((p[1:1 + nv].tolist(), tab))
    F, pool = encode_filters(kinds, pays)
    ref = gpu_search(idx, w.Q, F, pool, 10, 48)
    _say("table filters through the server")
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=48), max_batch=8, n_streams=2, max_wait_us=50)
    try:
        t = jag.jag_server_submit(s, w.Q, F, pool)
        mix = _collect(s, t)
        alone = []
        for i in range(0, w.nq, 5):
            f = F[i:i + 1].copy()
            p = pool[f[0, 4]:f[0, 4] + f[0, 5]].copy() if f[0, 0] == FILTER_TABLE else np.zeros(1, np.int32)
            f[0, 4] = 0
            alone.append((i, _collect(s, jag.jag_server_submit(s, w.Q[i:i + 1], f, p))[0]))
    finally:
        jag.jag_server_stop(s)
    for q, (ids, d, c, lat) in enumerate(mix):
        assert np.array_equal(ids, ref["ids"][q]) and c == ref["count"][q], q
    for i, (ids, d, c, lat) in alone:
        assert np.array_equal(ids, ref["ids"][i]) and c == ref["count"][i], i


def test_failed_batch_stops_the_server_instead_of_hanging(mixed_world, monkeypatch):
    """A batch whose completion check reports a device error (forced from the
    host by the test hook; the device work itself finishes normally) stops the
    server: drain and poll report JAG_EDEVICE, submit refuses new requests,
    stop returns, and nothing waits forever."""
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    monkeypatch.setenv("JAG_SERVER_TEST_FAIL_BATCH", "2")
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=32), max_batch=4, n_streams=1, max_wait_us=0)
    monkeypatch.delenv("JAG_SERVER_TEST_FAIL_BATCH")
    try:
        t = jag.jag_server_submit(s, w.Q[:40], w.F[:40], w.pool)
        t0 = time.time()
        with pytest.raises(jag.JagError) as e:
            jag.jag_server_drain(s)
        assert e.value.status == jag.JAG_EDEVICE
        assert time.time() - t0 < 30
        first = [jag.jag_server_poll(s, int(x)) for x in t[:4]]  # batch 1 completed
        assert all(r is not None for r in first)
        for x in t[4:8]:  # batch 2 failed
            with pytest.raises(jag.JagError) as e:
                jag.jag_server_poll(s, int(x))
            assert e.value.status == jag.JAG_EDEVICE
        with pytest.raises(jag.JagError) as e:
            jag.jag_server_submit(s, w.Q[:1], w.F[:1], w.pool)
        assert e.value.status == jag.JAG_EDEVICE
    finally:
        jag.jag_server_stop(s)
    _say("failed batch reported, server stopped")
