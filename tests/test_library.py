"""CPU checks of the product library: it loads, exports every entry point the
header declares, rejects bad arguments, and its host-only graph builder
produces a valid, deterministic, useful graph."""
import collections
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_10258_amd import jag
from workloads import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "jag.h")).read()
    return sorted(set(re.findall(r"^\s*(?:jag_status|void|const char \*)\s*(jag_\w+)\s*\(", src, re.M)))


def test_library_exports_every_header_symbol():
    L = jag.lib()
    syms = _header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) <= set(jag.exported_symbols()) | {"jag_free"}
    assert b"gfx950" in L.jag_version()


def test_library_shares_one_hip_runtime_with_torch():
    """Loading the library before anything imports torch must not map a second
    HIP runtime beside PyTorch's (with two, PyTorch finds no device)."""
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r)\n"
            "from paper_2602_10258_amd import jag\n"
            "jag.lib()\n"
            "import torch\n"
            "m = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(m), sorted(m))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[0] == "1", out.stdout


def test_build_graph_rejects_bad_arguments():
    X = np.zeros((10, 4), np.float32)
    with pytest.raises(jag.JagError) as e:
        jag.jag_build_graph(X, R=0)
    assert e.value.status == jag.JAG_EINVAL
    with pytest.raises(jag.JagError):  # thresholds name a scalar attribute that is absent
        jag.jag_build_graph(X, R=4, thresholds=[(jag.ATTR_SCALAR, 0.5)])
    with pytest.raises(jag.JagError):  # unsorted label rows
        jag.jag_build_graph(X, label_off=np.array([0, 2] + [2] * 9), labels=np.array([3, 1]),
                            vocab=4, R=4, thresholds=[(jag.ATTR_LABELS, 0.0)])
    with pytest.raises(jag.JagError):  # label outside the vocabulary
        jag.jag_build_graph(X, label_off=np.arange(11), labels=np.full(10, 9), vocab=4, R=4,
                            thresholds=[(jag.ATTR_LABELS, 0.0)])
    Xn = X.copy()
    Xn[3, 2] = np.nan
    with pytest.raises(jag.JagError):
        jag.jag_build_graph(Xn, R=4, thresholds=[(jag.ATTR_SCALAR, 1.0)], scalar=np.zeros(10))


def _reach(adj, s):
    seen = {s}
    dq = collections.deque([s])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if v >= 0 and v not in seen:
                seen.add(int(v))
                dq.append(int(v))
    return len(seen)


def test_host_builder_structure_determinism_and_recall():
    """The product builder is parity unpinned (no reference graph): structure,
    determinism across thread counts, and recall through the oracle's search."""
    w = make_config("c1")
    kw = dict(label_off=w.loff, labels=w.lab, vocab=8, R=32, L_build=64,
              thresholds=[(jag.ATTR_LABELS, 1.0), (jag.ATTR_LABELS, 0.0)], seed=0)
    adj, entry = jag.jag_build_graph(w.X, n_threads=8, **kw)
    adj1, entry1 = jag.jag_build_graph(w.X, n_threads=1, **kw)
    assert entry == entry1 and np.array_equal(adj, adj1)
    deg = (adj >= 0).sum(1)
    assert deg.max() <= 32 and deg.min() >= 1
    for i in range(0, w.n, 101):
        row = adj[i][:deg[i]]
        assert i not in row.tolist() and len(set(row.tolist())) == deg[i]
        assert np.all(adj[i][deg[i]:] == -1)
    assert _reach(adj, entry) >= 0.999 * w.n
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10, nthreads=4)
    r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, 64, 10)
    assert np.nanmean(O.recall_at_k(r.ids, gi, gd, nv, 10)) >= 0.95


def test_host_builder_range_and_labelsets():
    w = make_config("c4", n=3000, nq=60)
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=8,
                                     R=24, thresholds=[(jag.ATTR_SCALAR, 1.0), (jag.ATTR_SCALAR, 0.01),
                                                       (jag.ATTR_SCALAR, 0.0), (jag.ATTR_LABELS, 0.0)],
                                     seed=1)
    assert (adj >= 0).sum(1).max() <= 24
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10)
    r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, 128, 10)
    assert np.nanmean(O.recall_at_k(r.ids, gi, gd, nv, 10)) >= 0.9


def test_weighted_label_distance_builds_navigable_label_graphs():
    """Zipf label sets over a large vocabulary (the shape of the subset/Boolean
    workload at 20k points): graphs built with the frequency-weighted label
    distance (App. D.3) are searched to far higher recall than with |a XOR b|,
    through the oracle's search; the weighted build is deterministic."""
    w = make_config("c3", n=20000, nq=200)
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10, nthreads=8)
    rec = {}
    for kind in (jag.ATTR_LABELS, jag.ATTR_LABELS_WEIGHTED):
        kw = dict(label_off=w.loff, labels=w.lab, vocab=w.vocab, R=32, L_build=64,
                  thresholds=[(kind, 1.0), (kind, 0.01), (kind, 0.0)], seed=0)
        adj, entry = jag.jag_build_graph(w.X, n_threads=8, **kw)
        if kind == jag.ATTR_LABELS_WEIGHTED:
            adj1, entry1 = jag.jag_build_graph(w.X, n_threads=3, **kw)
            assert entry == entry1 and np.array_equal(adj, adj1)
            assert (adj >= 0).sum(1).max() <= 32
        r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, 64, 10, nthreads=8)
        rec[kind] = float(np.nanmean(O.recall_at_k(r.ids, gi, gd, nv, 10)))
    # measured: 0.40 with |a XOR b|, 0.79 weighted (R = 32, beam 64)
    assert rec[jag.ATTR_LABELS_WEIGHTED] >= 0.7, rec
    assert rec[jag.ATTR_LABELS_WEIGHTED] >= rec[jag.ATTR_LABELS] + 0.25, rec


def test_host_builder_weight_entries_reach_the_threshold_limits():
    """The product builder's Weight-JAG entries at their two limits give
    exactly its Threshold-JAG graphs (w = 0 -> 100 %, huge w -> 0)."""
    rng = np.random.default_rng(12)
    n = 2000
    X = rng.normal(0, 1, size=(n, 8)).astype(np.float32)
    scal = rng.integers(0, 60, size=n).astype(np.int32)
    W = jag.THRESHOLD_WEIGHT
    kw = dict(scalar=scal, R=12, L_build=24, seed=4, n_threads=4)
    g0, e0 = jag.jag_build_graph(X, thresholds=[(jag.ATTR_SCALAR | W, 0.0)], **kw)
    gi, ei = jag.jag_build_graph(X, thresholds=[(jag.ATTR_SCALAR, 1.0)], **kw)
    assert e0 == ei and np.array_equal(g0, gi)
    gw, ew = jag.jag_build_graph(X, thresholds=[(jag.ATTR_SCALAR | W, 1e6)], **kw)
    gz, ez = jag.jag_build_graph(X, thresholds=[(jag.ATTR_SCALAR, 0.0)], **kw)
    assert ew == ez and np.array_equal(gw, gz)
    with pytest.raises(jag.JagError):
        jag.jag_build_graph(X, thresholds=[(jag.ATTR_SCALAR | 0x200, 0.0)], **kw)


def test_weight_jag_builds_a_searchable_range_graph():
    """Weight-JAG with the paper's range weight list {0, 10h, 1000h} gives a
    graph the oracle's search answers range queries on well."""
    w = make_config("c2", n=20000, nq=200)
    W = jag.THRESHOLD_WEIGHT
    adj, entry = jag.jag_build_graph(w.X, scalar=w.scalar, R=32, L_build=64, n_threads=8,
                                     thresholds=[(jag.ATTR_SCALAR | W, 0.0), (jag.ATTR_SCALAR | W, 10.0),
                                                 (jag.ATTR_SCALAR | W, 1000.0)], seed=0)
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10, nthreads=8)
    r = O.search(w.X, adj, entry, A, w.Q, w.F, w.pool, 128, 10, nthreads=8)
    rec = float(np.nanmean(O.recall_at_k(r.ids, gi, gd, nv, 10)))
    assert rec >= 0.9, rec


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding passes by pointer has the header's size and
    field offsets (the header compiled by the host C compiler)."""
    import ctypes as C
    import json
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    structs = {"jag_search_params": jag.jag_search_params, "jag_index_info": jag.jag_index_info,
               "jag_server_params": jag.jag_server_params, "jag_server_stats": jag.jag_server_stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "jag.h"', "int main(void) {",
             'printf("{");']
    first = True
    for name, cls in structs.items():
        for field, _ in cls._fields_:
            sep = "" if first else ","
            first = False
            lines.append(f'printf("{sep}\\"{name}.{field}\\": %zu", offsetof({name}, {field}));')
        lines.append(f'printf(",\\"{name}\\": %zu", sizeof({name}));')
    lines += ['printf("}\\n");', "return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    want = json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)
    for name, cls in structs.items():
        assert C.sizeof(cls) == want[name], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == want[f"{name}.{field}"], (name, field)


def test_gather_ceiling_rejects_bad_arguments():
    """Argument checks happen before any device call (no GPU needed)."""
    import ctypes as C
    L = jag.lib()
    out = C.c_double(-1.0)
    fake = C.c_void_p(4096)  # never dereferenced: the checks fail first
    for args in [(None, 1 << 30, 192, 64, 10, 1), (fake, 1 << 30, 100, 64, 10, 1), (fake, 1 << 30, 192, 0, 10, 1),
                 (fake, 1 << 30, 192, 64, 0, 1), (fake, 1 << 30, 192, 64, 10, 0), (fake, 1000, 192, 64, 10, 1),
                 (fake, 1 << 30, 448, 64, 10, 1)]:  # 448 is no multiple of 8 lanes x 16 bytes
        st = L.jag_gather_ceiling(args[0], *args[1:], None, C.byref(out))
        assert st == jag.JAG_EINVAL, args
    assert out.value == -1.0


def test_predictor_targets_take_the_recall_plateau_of_unreachable_queries():
    """Target = smallest ladder index reaching recall 0.95; a query that never
    reaches it gets the widest index, or with the plateau rule the smallest
    index where its recall peaks; queries without valid items get index 0."""
    from paper_2602_10258_amd.predictor import targets_from
    ex = np.array([[1, 2], [3, 4], [5, 6], [7, 8]], np.int32)
    cnt = np.array([2, 2, 2, 0])
    ids = np.array([[[1, 9], [3, 9], [5, 9], [0, 0]],
                    [[1, 2], [3, 9], [9, 9], [0, 0]],
                    [[1, 2], [3, 4], [5, 6], [0, 0]],
                    [[1, 2], [3, 9], [5, 6], [0, 0]]], np.int32)  # 4 levels x 4 queries x k
    t, r = targets_from(ids, ex, cnt, 2)
    assert t.tolist() == [1, 2, 2, 0] and r.tolist() == [True, True, True, True]
    ids2 = ids.copy()
    ids2[:, 1, 1] = 9   # query 1 never finds label 4: peak (1 hit) first at level 0
    ids2[:, 2, :] = [[5, 9], [9, 9], [5, 9], [5, 9]]  # query 2 peaks at 1 hit, first at level 0
    t, r = targets_from(ids2, ex, cnt, 2, unreachable="plateau")
    assert t.tolist() == [1, 0, 0, 0] and r.tolist() == [True, False, False, True]
    t, r = targets_from(ids2, ex, cnt, 2)  # default: unreachable queries train toward the widest beam
    assert t.tolist() == [1, 3, 3, 0] and r.tolist() == [True, False, False, True]
