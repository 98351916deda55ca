"""Pins for the oracle's filter and attribute distances (Sections 3.1 and 3.2)."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import FILTER_BOOLEAN, FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_TABLE, encode_filters

HERE = os.path.dirname(os.path.abspath(__file__))


def _attrs_from_sets(sets, scalars=None):
    n = len(sets)
    loff = np.zeros(n + 1, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in sorted(s)], dtype=np.int32)
    if lab.size == 0:
        lab = np.zeros(1, dtype=np.int32)
    sc = None if scalars is None else np.asarray(scalars, dtype=np.int32)
    return O.Attrs(n, sc, loff, lab)


def _parse_bool(s):
    clauses = []
    for cl in s.split("|"):
        cl = cl.strip().strip("()")
        lits = []
        for t in cl.split("&"):
            t = t.strip()
            lits.append(~int(t[1:]) if t.startswith("~") else int(t))
        clauses.append(lits)
    return clauses


def _golden_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "dist_f_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([c.strip() for c in line.split(";")])
    return rows


def _labels(s):
    return set(int(v) for v in s.strip("{}").split(",") if v.strip())


def _golden_case(row):
    typ, filt, attr, expect = row[0], row[1], row[2], float(row[3])
    if typ == "range":
        lo, hi = (int(v) for v in filt.strip("[]").split(","))
        F, pool = encode_filters([FILTER_RANGE], [(lo, hi)])
        A = _attrs_from_sets([set()], scalars=[int(attr)])
    else:
        A = _attrs_from_sets([_labels(attr)])
        if typ == "label":
            F, pool = encode_filters([FILTER_LABEL], [int(filt)])
        elif typ == "subset":
            F, pool = encode_filters([FILTER_SUBSET], [sorted(_labels(filt))])
        else:
            F, pool = encode_filters([FILTER_BOOLEAN], [_parse_bool(filt)])
    return A, F, pool, expect


def test_golden_fixture_parses():
    rows = _golden_rows()
    assert len(rows) == 19
    assert {r[0] for r in rows} == {"label", "range", "subset", "boolean"}


@pytest.mark.parametrize("case", range(19))
def test_dist_f_hand_worked(case):
    row = _golden_rows()[case]
    A, F, pool, expect = _golden_case(row)
    got = O.dist_f(A, [0], F, [0], pool)[0]
    assert got == expect, (row, got)


def _g(kind, payload, labels, scalar):
    """The match function g(a, f) of Section 2, written as plain set logic."""
    if kind == FILTER_LABEL:
        return payload in labels
    if kind == FILTER_RANGE:
        return payload[0] <= scalar <= payload[1]
    if kind == FILTER_SUBSET:
        return set(payload) <= labels
    return any(all((l in labels) if l >= 0 else ((~l) not in labels) for l in cl) for cl in payload)


def test_validity_axiom_random():
    """dist_F(a, f) = 0 exactly when g(a, f) = 1 (Section 3.1, validity)."""
    rng = np.random.default_rng(5)
    n = 300
    sets = [set(rng.choice(12, size=rng.integers(0, 6), replace=False).tolist()) for _ in range(n)]
    scal = rng.integers(0, 50, size=n)
    A = _attrs_from_sets(sets, scal)
    kinds, pays = [], []
    for _ in range(200):
        t = int(rng.integers(0, 4))
        if t == FILTER_LABEL:
            p = int(rng.integers(0, 12))
        elif t == FILTER_RANGE:
            lo = int(rng.integers(0, 50))
            p = (lo, lo + int(rng.integers(0, 10)))
        elif t == FILTER_SUBSET:
            p = rng.choice(12, size=rng.integers(1, 4), replace=False).tolist()
        else:
            p = [[int(v) if rng.random() < 0.7 else ~int(v)
                  for v in rng.choice(12, size=rng.integers(1, 4), replace=False)]
                 for _ in range(rng.integers(1, 4))]
        kinds.append(t)
        pays.append(p)
    F, pool = encode_filters(kinds, pays)
    items = np.repeat(np.arange(n), len(kinds))
    fidx = np.tile(np.arange(len(kinds)), n)
    df = O.dist_f(A, items, F, fidx, pool)
    for j in range(len(items)):
        i, f = int(items[j]), int(fidx[j])
        assert (df[j] == 0) == _g(kinds[f], pays[f], sets[i], int(scal[i])), (i, kinds[f], pays[f])
        assert df[j] >= 0


def test_boolean_dist_is_min_flips_bruteforce():
    """Boolean dist_F = fewest bit flips that satisfy f, by enumerating all 2^m assignments."""
    rng = np.random.default_rng(11)
    m = 8
    for trial in range(150):
        ncl = int(rng.integers(1, 4))
        prog = []
        for _ in range(ncl):
            vs = rng.choice(m, size=rng.integers(1, 4), replace=True)  # duplicates allowed
            prog.append([int(v) if rng.random() < 0.6 else ~int(v) for v in vs])
        F, pool = encode_filters([FILTER_BOOLEAN], [prog])
        a = set(rng.choice(m, size=rng.integers(0, m), replace=False).tolist())
        A = _attrs_from_sets([a])
        got = O.dist_f(A, [0], F, [0], pool)[0]
        best = None
        for bits in itertools.product([0, 1], repeat=m):
            s = {i for i in range(m) if bits[i]}
            if _g(FILTER_BOOLEAN, prog, s, 0):
                h = len(s ^ a)
                best = h if best is None else min(best, h)
        if best is None:
            assert got == 4294967295.0
        else:
            assert got == best, (prog, a, got, best)


def test_subset_dist_counts_missing_labels():
    """|f minus a| against independent set arithmetic over random sets."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        a = set(rng.choice(20, size=rng.integers(0, 10), replace=False).tolist())
        f = rng.choice(20, size=rng.integers(1, 6), replace=False).tolist()
        A = _attrs_from_sets([a])
        F, pool = encode_filters([FILTER_SUBSET], [f])
        assert O.dist_f(A, [0], F, [0], pool)[0] == len(set(f) - a)


def test_attribute_distance_validity_and_capping():
    """dist_A = 0 exactly for equal attributes; the cap max(dist_A - t, 0) (Section 3.2)."""
    rng = np.random.default_rng(7)
    n = 200
    sets = [set(rng.choice(6, size=rng.integers(0, 4), replace=False).tolist()) for _ in range(n)]
    scal = rng.integers(-20, 20, size=n)
    A = _attrs_from_sets(sets, scal)
    i1 = rng.integers(0, n, size=2000)
    i2 = rng.integers(0, n, size=2000)
    ds = O.dist_a(A, O.KIND_SCALAR, i1, i2, 0.0)
    dl = O.dist_a(A, O.KIND_LABELS, i1, i2, 0.0)
    for j in range(len(i1)):
        a, b = int(i1[j]), int(i2[j])
        assert (ds[j] == 0) == (scal[a] == scal[b])
        assert (dl[j] == 0) == (sets[a] == sets[b])
        assert dl[j] == len(sets[a] ^ sets[b])  # |a1 XOR a2|
        assert ds[j] == abs(int(scal[a]) - int(scal[b]))
    # t = +inf turns attribute order off entirely; t caps from below
    assert np.all(O.dist_a(A, O.KIND_SCALAR, i1, i2, np.inf) == 0)
    for t in (1.0, 3.0, 10.0):
        dt = O.dist_a(A, O.KIND_SCALAR, i1, i2, t)
        assert np.all(dt == np.maximum(ds - t, 0))
        assert np.all(dt <= ds)


def test_range_capped_dist_is_range_filter_distance():
    """max(|a_p - a_u| - t, 0) equals dist_F of a_u against the range [a_p - t, a_p + t]."""
    rng = np.random.default_rng(9)
    n = 400
    scal = rng.integers(0, 1000, size=n)
    A = _attrs_from_sets([set()] * n, scal)
    p = 17
    for t in (0, 5, 50):
        F, pool = encode_filters([FILTER_RANGE], [(int(scal[p]) - t, int(scal[p]) + t)])
        df = O.dist_f(A, np.arange(n), F, np.zeros(n, dtype=np.int32), pool)
        da = O.dist_a(A, O.KIND_SCALAR, np.full(n, p), np.arange(n), float(t))
        assert np.array_equal(df, da)


def test_weighted_label_distance_hand_worked():
    """Frequency-weighted label distance (App. D.3) on a five-item example
    worked by hand (tests/golden/dist_a_weighted_examples.txt)."""
    A = _attrs_from_sets([{0}, {0, 1}, {0, 2}, {0, 1, 2}, {3}])
    rows = []
    with open(os.path.join(HERE, "golden", "dist_a_weighted_examples.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                u, v, val = line.split()
                rows.append((int(u), int(v), float(val)))
    assert len(rows) == 6
    u = np.array([r[0] for r in rows])
    v = np.array([r[1] for r in rows])
    got = O.dist_a(A, O.KIND_LABELS_WEIGHTED, u, v, 0.0)
    np.testing.assert_allclose(got, [r[2] for r in rows], rtol=0, atol=1e-12)
    # symmetric; sharing a rarer label brings items closer than sharing a common one
    assert np.array_equal(got, O.dist_a(A, O.KIND_LABELS_WEIGHTED, v, u, 0.0))
    assert got[0] < got[2]
    # capping as for the other kinds
    capped = O.dist_a(A, O.KIND_LABELS_WEIGHTED, u, v, 1.0)
    np.testing.assert_allclose(capped, np.maximum(got - 1.0, 0.0), atol=1e-12)


def _table_filter(vars_, true_on):
    tab = np.zeros(1 << len(vars_), dtype=bool)
    tab[list(true_on)] = True
    return encode_filters([FILTER_TABLE], [(vars_, tab)])


def test_table_filter_hand_worked():
    """General Boolean filter (Section 3.1) given as a truth table over labels
    3, 1, 2 (assignment bit 0 = label 3, bit 1 = label 1, bit 2 = label 2),
    true on assignments 0b000, 0b101 and 0b111; distances worked by hand."""
    A = _attrs_from_sets([{1}, {3, 2}, set(), {1, 2}, {3}, {1, 2, 3}, {0}])
    F, pool = _table_filter([3, 1, 2], [0, 5, 7])
    d = O.dist_f(A, np.arange(7), F, np.zeros(7, dtype=np.int32), pool)
    # {1}: x=010 -> nearest 000 (1 flip); {3,2}: x=101 true; {}: true;
    # {1,2}: x=110 -> 111 (1); {3}: x=001 -> 000 or 101 (1); {1,2,3}: true;
    # {0}: label 0 is not a variable, x=000 true
    assert d.tolist() == [1, 0, 0, 1, 1, 0, 0]
    F, pool = _table_filter([3, 1, 2], [])
    assert np.all(O.dist_f(A, np.arange(7), F, np.zeros(7, dtype=np.int32), pool) == 2 ** 32 - 1)


def test_table_filter_equals_dnf_distance():
    """A DNF filter and its truth table give the same distance on every item
    (the DNF distance is pinned above by brute force over assignments)."""
    rng = np.random.default_rng(31)
    n = 300
    sets = [set(rng.choice(9, size=rng.integers(0, 6), replace=False).tolist()) for _ in range(n)]
    A = _attrs_from_sets(sets)
    for trial in range(40):
        vars_ = sorted(rng.choice(9, size=rng.integers(1, 7), replace=False).tolist())
        clauses = []
        for _ in range(rng.integers(1, 4)):
            m = rng.integers(1, len(vars_) + 1)
            lits = rng.choice(vars_, size=m, replace=False).tolist()
            clauses.append([int(l) if rng.random() < 0.6 else ~int(l) for l in lits])
        # truth table by evaluating the DNF on each assignment of the variables
        tab = []
        for x in range(1 << len(vars_)):
            held = {v for b, v in enumerate(vars_) if (x >> b) & 1}
            tab.append(any(all((l in held) if l >= 0 else (~l not in held) for l in cl) for cl in clauses))
        Fd, pd = encode_filters([FILTER_BOOLEAN], [clauses])
        Ft, pt = encode_filters([FILTER_TABLE], [(vars_, np.array(tab))])
        idx = np.arange(n)
        dd = O.dist_f(A, idx, Fd, np.zeros(n, dtype=np.int32), pd)
        dt = O.dist_f(A, idx, Ft, np.zeros(n, dtype=np.int32), pt)
        assert np.array_equal(dd, dt), (trial, vars_, clauses)


def test_table_filter_validity_in_bruteforce():
    """The exact k-NN's validity test for table filters (the function's value)
    agrees with distance zero."""
    from workloads import make_config
    w = make_config("bool15", n=3000, nq=12)
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, 10)
    for q in range(w.nq):
        d = O.dist_f(A, np.arange(w.n), w.F, np.full(w.n, q, dtype=np.int32), w.pool)
        assert nv[q] == int((d == 0).sum())
        got = gi[q][gi[q] >= 0]
        assert np.all(d[got] == 0)
