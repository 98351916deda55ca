"""GPU tests of the server's slot admission (resident waves that take one
request at a time): answers equal to the oracle and to a direct search,
alone and in the mix, with truth-table filters, the learned one-pass beam,
fewer waves than requests, restarts after the waves' idle exit, concurrent
submitters, budgets and the failure path."""
import sys
import threading
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag

from .parity import compare_strict, lane_order
from .test_gpu_search import _index, gpu_search
from .test_gpu_serving import _collect, _rows

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _same(res, ref, order):
    for (ids, d, c, lat), q in zip(res, order):
        assert c == ref["count"][q] and np.array_equal(ids, ref["ids"][q]), q
        assert np.array_equal(d.view(np.uint32), ref["d2"][q].view(np.uint32)), q


@pytest.mark.parametrize("store", [jag.STORE_F32, jag.STORE_BF16])
def test_slots_match_oracle_alone_and_in_mix(mixed_world, store):
    w, A, adj, entry = mixed_world
    _say("slot server alone vs mix, store", store)
    quant = store != jag.STORE_F32
    idx = _index(w, adj, entry, store=store, keep_f32=True)
    rr = 4 if quant else 0
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 48, rerank_mult=rr)
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=48, rerank_mult=rr), slot_admission=True)
    try:
        t_mix = np.concatenate([jag.jag_server_submit(s, w.Q[i::4], w.F[i::4], w.pool) for i in range(4)])
        order = np.concatenate([np.arange(i, w.nq, 4) for i in range(4)])
        mix = _collect(s, t_mix)
        alone = []
        for i in range(0, w.nq, 7):
            f, p = _rows(w.F, w.pool, i)
            alone.append((i, _collect(s, jag.jag_server_submit(s, w.Q[i:i + 1], f, p))[0]))
        st = jag.jag_server_stats_get(s)
    finally:
        jag.jag_server_stop(s)
    _same(mix, ref, order)
    _same([r for _, r in alone], ref, [i for i, _ in alone])
    # the server's answers against the oracle in the kernel's summation order
    base = O.bf16_decode(O.bf16_encode(w.X)) if quant else w.X
    orc = O.search(base, adj, entry, A, w.Q, w.F, w.pool, 48, 10, rerank=w.X if quant else None,
                   rerank_mult=4, nthreads=8, contract=lane_order(store, w.d))
    got = sorted(zip(order, mix), key=lambda x: x[0])
    compare_strict(np.stack([r[0] for _, r in got]), np.stack([r[1] for _, r in got]),
                   np.array([r[2] for _, r in got]), orc, f"slot server store={store} (contract)")
    assert st["completed"] == w.nq + len(alone)
    assert st["p99_us"] >= st["p50_us"] > 0 and st["batches"] >= 1
    assert st["resident_capacity"] > 0 and st["device_bytes"] > 0
    _say(st)


def test_slots_with_few_waves_and_learned_beam(mixed_world):
    """Eight waves for 4 x nq requests (most wait in the ring for a free wave),
    and the learned beam in one pass: the same answers as the direct search."""
    w, A, adj, entry = mixed_world
    from .test_gpu_learned import _params
    idx = _index(w, adj, entry, store=jag.STORE_BF16, keep_f32=True)
    jag.jag_set_predictor(idx, _params(41, scale=0.4), np.array([10, 16, 24, 40, 64], np.int32), 2.5)
    for learned in (0, 1):
        sp = jag.SearchParams(L=40, learned=learned, rerank_mult=4)
        ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 40, learned=learned, rerank_mult=4, single_pass=1)
        s = jag.jag_server_start(idx, 10, sp, slot_admission=True, max_inflight=8)
        try:
            t = jag.jag_server_submit(s, np.tile(w.Q, (4, 1)), np.tile(w.F, (4, 1)), w.pool)
            jag.jag_server_drain(s)
            res = _collect(s, t)
            st = jag.jag_server_stats_get(s)
        finally:
            jag.jag_server_stop(s)
        _same(res, ref, np.tile(np.arange(w.nq), 4))
        assert st["completed"] == 4 * w.nq and st["max_inflight_seen"] > 8
        _say("learned", learned, "8 waves:", {k: st[k] for k in ("batches", "p50_us", "p99_us", "device_bytes")})


def test_slots_restart_after_idle_exit_with_table_filters():
    """Truth-table filters (their tables copied by the wave that runs them) and
    plain label filters; between the two rounds of requests the waves leave
    after their idle interval and the server starts them again."""
    from workloads import FILTER_LABEL, FILTER_TABLE, encode_filters
    from .test_gpu_table_filters import _bool_world
    w, A, adj, entry = _bool_world(10, nq=64, seed=7)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=w.vocab)
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
    _say("table filters through the slot server")
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=48), slot_admission=True)
    try:
        first = _collect(s, jag.jag_server_submit(s, w.Q, F, pool))
        time.sleep(0.1)  # ten idle intervals: the waves have left
        alone = []
        for i in range(0, w.nq, 5):
            f = F[i:i + 1].copy()
            p = pool[f[0, 4]:f[0, 4] + f[0, 5]].copy() if f[0, 0] == FILTER_TABLE else np.zeros(1, np.int32)
            f[0, 4] = 0
            alone.append((i, _collect(s, jag.jag_server_submit(s, w.Q[i:i + 1], f, p))[0]))
        st = jag.jag_server_stats_get(s)
    finally:
        jag.jag_server_stop(s)
    _same(first, ref, np.arange(w.nq))
    _same([r for _, r in alone], ref, [i for i, _ in alone])
    assert st["batches"] >= 2, st  # launched again after the idle exit
    _say("launches", st["batches"])


def test_slots_concurrent_submitters(mixed_world):
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 40)
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=40), slot_admission=True)
    got = {}

    def client(j):
        for i in range(j, w.nq, 4):
            f, p = _rows(w.F, w.pool, i)
            got[i] = jag.jag_server_submit(s, w.Q[i:i + 1], f, p)[0]

    try:
        th = [threading.Thread(target=client, args=(j,)) for j in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        res = _collect(s, [got[i] for i in range(w.nq)])
    finally:
        jag.jag_server_stop(s)
    _same(res, ref, np.arange(w.nq))


def test_slots_budget_and_parameters(mixed_world):
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    with pytest.raises(jag.JagError) as e:
        jag.jag_server_start(idx, 10, jag.SearchParams(L=32), slot_admission=True, hbm_budget_bytes=1000)
    assert e.value.status == jag.JAG_EUNSUPPORTED
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=32), slot_admission=True, max_inflight=3,
                             queue_capacity=10)
    try:
        st = jag.jag_server_stats_get(s)
        with pytest.raises(jag.JagError) as e:
            jag.jag_server_submit(s, w.Q[:11], w.F[:11], w.pool)
        assert e.value.status == jag.JAG_EBUSY
        t = jag.jag_server_submit(s, w.Q[:10], w.F[:10], w.pool)
        jag.jag_server_drain(s)
        assert len(_collect(s, t)) == 10
    finally:
        jag.jag_server_stop(s)
    # three waves: a query copy and a table copy each, plus the counters
    per_wave = (4 * w.d + 255) // 256 * 256 + (1 << 15)
    assert st["device_bytes"] == 3 * per_wave + 512


def test_slots_failed_launch_stops_the_server(mixed_world, monkeypatch):
    """The end of the first launch of waves reported as a device error (forced
    from the host by the test hook once the waves have left normally): the
    requests answered before stay available, submit refuses new requests and
    stop returns."""
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    monkeypatch.setenv("JAG_SERVER_TEST_FAIL_BATCH", "1")
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=32), slot_admission=True)
    monkeypatch.delenv("JAG_SERVER_TEST_FAIL_BATCH")
    try:
        t = jag.jag_server_submit(s, w.Q[:40], w.F[:40], w.pool)
        jag.jag_server_drain(s)
        t0 = time.time()
        while True:  # the waves leave after their idle interval; the hook then fires
            try:
                jag.jag_server_submit(s, w.Q[:1], w.F[:1], w.pool)
            except jag.JagError as e:
                assert e.status == jag.JAG_EDEVICE
                break
            assert time.time() - t0 < 30, "the failure was never reported"
            time.sleep(0.02)
        assert all(jag.jag_server_poll(s, int(x)) is not None for x in t)
    finally:
        jag.jag_server_stop(s)
    _say("failed launch reported, server stopped")


def test_slots_ring_wraps_with_few_waves(mixed_world):
    """Eight waves and 3,200 requests: the 1,024-slot ring is reused three
    times over (a slot is written again only after its answer was
    collected), and every answer is the direct search's."""
    w, A, adj, entry = mixed_world
    idx = _index(w, adj, entry)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 32)
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=32), slot_admission=True, max_inflight=8)
    try:
        t = jag.jag_server_submit(s, np.tile(w.Q, (20, 1)), np.tile(w.F, (20, 1)), w.pool)
        jag.jag_server_drain(s)
        res = _collect(s, t)
        st = jag.jag_server_stats_get(s)
    finally:
        jag.jag_server_stop(s)
    _same(res, ref, np.tile(np.arange(w.nq), 20))
    assert st["completed"] == 20 * w.nq and st["max_inflight_seen"] <= 1024
    _say("ring reused:", {k: st[k] for k in ("batches", "max_inflight_seen", "p99_us")})


def test_slots_table_area_wraps_with_wide_tables():
    """Fifteen-variable tables (32 KiB each) in numbers that overflow the
    server's 8 MiB host table area: publishing waits for answered requests to
    free their tables, the area wraps around, and every answer is the direct
    search's."""
    from .test_gpu_table_filters import _bool_world
    w, A, adj, entry = _bool_world(15, nq=24)
    idx = jag.jag_build_from_graph(w.X, adj, entry, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    ref = gpu_search(idx, w.Q, w.F, w.pool, 10, 48)
    reps = 40  # 960 tables, 30 MiB
    F = np.tile(w.F, (reps, 1))
    _say("wide tables through the slot server:", F.shape[0])
    s = jag.jag_server_start(idx, 10, jag.SearchParams(L=48), slot_admission=True)
    try:
        res = _collect(s, jag.jag_server_submit(s, np.tile(w.Q, (reps, 1)), F, w.pool), timeout=120.0)
    finally:
        jag.jag_server_stop(s)
    _same(res, ref, np.tile(np.arange(w.nq), reps))
