"""Seeded generators for the five workload shapes of the filtered-search study.

Every array comes from ``numpy.random.default_rng(seed)``, so the same call
gives the same bytes on any machine with the same numpy.  Shapes follow the
paper's workloads (Section 4 and Appendix D.2: label, range, subset and
Boolean filters over clustered embeddings); the paper's datasets themselves
are not used.

Filter records are int32 rows ``(type, label, lo, hi, off, len)``:

* LABEL   (0): ``label`` is the required label (membership in the item's
  label set; for single-label items this is label equality).
* RANGE   (1): inclusive ``[lo, hi]`` on the item's scalar attribute.
* SUBSET  (2): ``pool[off:off+len]`` are labels that must all be present.
* BOOLEAN (3): ``pool[off:off+len]`` is a DNF program
  ``ncl, nlit_1, lit..., nlit_2, lit..., ...`` where a literal ``l >= 0``
  asks for label ``l`` and ``l < 0`` asks for the absence of label ``~l``.
* TABLE   (4): a general Boolean function of up to 15 labels,
  ``pool[off:off+len] = nvar, var_0..var_{nvar-1}, w_0..w_{W-1}``: the item's
  assignment x has bit i set when it holds label ``var_i``, and the function
  is true on x when bit ``x % 32`` of word ``w_{x // 32}`` is set
  (W = ceil(2^nvar / 32)).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_BOOLEAN, FILTER_TABLE = 0, 1, 2, 3, 4
RANGE_DOMAIN = 1_000_000  # scalar attributes are uniform over [0, 10^6)

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "bool15")


@dataclass
class Workload:
    name: str
    X: np.ndarray                       # float32 [n, d]
    Q: np.ndarray                       # float32 [nq, d]
    F: np.ndarray                       # int32 [nq, 6] filter records
    pool: np.ndarray                    # int32 [*] subset labels / DNF programs
    scalar: Optional[np.ndarray] = None  # int32 [n]
    loff: Optional[np.ndarray] = None    # int64 [n+1] CSR offsets of label sets
    lab: Optional[np.ndarray] = None     # int32 [nnz] sorted distinct labels per item
    vocab: int = 0
    k: int = 10
    R: int = 32
    L: int = 64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def nq(self) -> int:
        return self.Q.shape[0]


def mixture(rng: np.random.Generator, n: int, d: int, clusters: int,
            centers: Optional[np.ndarray] = None, center_std: float = 4.0,
            sigma: float = 1.0, chunk: int = 1 << 18):
    """Equal-weight Gaussian mixture: centres ~ N(0, center_std^2), spread sigma."""
    if centers is None:
        centers = rng.normal(0.0, center_std, size=(clusters, d))
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a = rng.integers(0, clusters, size=e - s)
        X[s:e] = (centers[a] + rng.normal(0.0, sigma, size=(e - s, d))).astype(np.float32)
    return X, centers


def _zipf_p(vocab: int, s: float) -> np.ndarray:
    r = np.arange(1, vocab + 1, dtype=np.float64)
    p = r ** (-s)
    return p / p.sum()


def zipf_label_sets(rng: np.random.Generator, n: int, vocab: int, lo: int, hi: int,
                    s: float = 1.1):
    """Per item U{lo..hi} distinct labels drawn Zipf(s) over ``vocab`` ranks.

    Label id = rank - 1.  Duplicates are redrawn (first distinct draws are
    kept).  Returns CSR ``(loff int64[n+1], lab int32[nnz])`` with each row
    sorted ascending.
    """
    p = _zipf_p(vocab, s)
    cdf = np.cumsum(p)
    cnt = rng.integers(lo, hi + 1, size=n)
    width = 3 * hi + 4
    draws = np.searchsorted(cdf, rng.random((n, width)), side="right").astype(np.int32)
    draws = np.minimum(draws, vocab - 1)
    # first occurrence mask in draw order
    order = np.argsort(draws, axis=1, kind="stable")
    srt = np.take_along_axis(draws, order, axis=1)
    dup_sorted = np.zeros_like(srt, dtype=bool)
    dup_sorted[:, 1:] = srt[:, 1:] == srt[:, :-1]
    first = np.ones_like(draws, dtype=bool)
    np.put_along_axis(first, order, ~dup_sorted, axis=1)
    rank = np.cumsum(first, axis=1)
    keep = first & (rank <= cnt[:, None])
    got = keep.sum(axis=1)
    rows = []
    short = np.nonzero(got < cnt)[0]
    sets = [None] * n
    for i in short:  # rare: extend with further draws until enough distinct labels
        cur = list(dict.fromkeys(draws[i][first[i]].tolist()))
        while len(cur) < cnt[i]:
            v = int(min(np.searchsorted(cdf, rng.random(), side="right"), vocab - 1))
            if v not in cur:
                cur.append(v)
        sets[i] = sorted(cur[: cnt[i]])
    loff = np.zeros(n + 1, dtype=np.int64)
    lens = cnt.astype(np.int64)
    loff[1:] = np.cumsum(lens)
    lab = np.empty(int(loff[-1]), dtype=np.int32)
    vals = np.where(keep, draws, np.iinfo(np.int32).max)
    vals.sort(axis=1)
    ok = np.ones(n, dtype=bool)
    ok[short] = False
    idx_ok = np.nonzero(ok)[0]
    # rows with enough draws: the first cnt sorted kept values
    for start in range(0, len(idx_ok), 1 << 16):
        ii = idx_ok[start:start + (1 << 16)]
        v = vals[ii]
        c = cnt[ii]
        m = np.arange(v.shape[1])[None, :] < c[:, None]
        lab_pos = loff[ii][:, None] + np.arange(v.shape[1])[None, :]
        lab[lab_pos[m]] = v[m]
    for i in short:
        lab[loff[i]:loff[i + 1]] = sets[i]
    del rows
    return loff, lab


def range_filters(rng: np.random.Generator, nq: int, sel_lo: float = 1e-4,
                  sel_hi: float = 1.0, domain: int = RANGE_DOMAIN):
    """Ranges whose width gives a log-uniform selectivity over [sel_lo, sel_hi]."""
    s = 10.0 ** rng.uniform(np.log10(sel_lo), np.log10(sel_hi), size=nq)
    w = np.maximum(1, np.rint(s * domain)).astype(np.int64)
    w = np.minimum(w, domain)
    lo = (rng.random(nq) * (domain - w + 1)).astype(np.int64)
    lo = np.minimum(lo, domain - w)
    hi = lo + w - 1
    return lo.astype(np.int32), hi.astype(np.int32)


def encode_filters(kinds, payloads):
    """Build (F int32[nq,6], pool int32[*]) from per-query python descriptions.

    kinds[i] in {0,1,2,3,4}; payloads[i] is: label (int) | (lo, hi) |
    list of labels | list of clauses, each a list of literals |
    (variable labels, truth table: bool array of length 2^nvar).
    """
    nq = len(kinds)
    F = np.zeros((nq, 6), dtype=np.int32)
    pool: list[int] = []
    for i, (t, p) in enumerate(zip(kinds, payloads)):
        F[i, 0] = t
        if t == FILTER_LABEL:
            F[i, 1] = int(p)
        elif t == FILTER_RANGE:
            F[i, 2], F[i, 3] = int(p[0]), int(p[1])
        elif t == FILTER_SUBSET:
            F[i, 4], F[i, 5] = len(pool), len(p)
            pool.extend(int(v) for v in p)
        elif t == FILTER_BOOLEAN:
            prog = [len(p)]
            for cl in p:
                prog.append(len(cl))
                prog.extend(int(v) for v in cl)
            F[i, 4], F[i, 5] = len(pool), len(prog)
            pool.extend(prog)
        elif t == FILTER_TABLE:
            vars_, table = p
            table = np.asarray(table, dtype=bool)
            nv = len(vars_)
            assert table.size == 1 << nv
            by = np.packbits(table, bitorder="little")  # bit j of byte b = table[8b + j]
            by = np.concatenate([by, np.zeros((-len(by)) % 4, dtype=np.uint8)])
            words = by.view("<u4")
            prog = [nv] + [int(v) for v in vars_] + words.view(np.int32).tolist()
            F[i, 4], F[i, 5] = len(pool), len(prog)
            pool.extend(prog)
        else:
            raise ValueError(f"unknown filter type {t}")
    return F, np.asarray(pool if pool else [0], dtype=np.int32)


def _zipf_draw(rng, vocab, size, s=1.1):
    cdf = np.cumsum(_zipf_p(vocab, s))
    return np.minimum(np.searchsorted(cdf, rng.random(size), side="right"), vocab - 1)


def _distinct_zipf(rng, vocab, m, s=1.1):
    out: list[int] = []
    while len(out) < m:
        v = int(_zipf_draw(rng, vocab, 1, s)[0])
        if v not in out:
            out.append(v)
    return out


def _subset_and_bool_queries(rng, nq_subset, nq_bool, vocab, max_subset=3):
    kinds, pays = [], []
    for _ in range(nq_subset):
        m = int(rng.integers(1, max_subset + 1))
        kinds.append(FILTER_SUBSET)
        pays.append(sorted(_distinct_zipf(rng, vocab, m)))
    for _ in range(nq_bool):
        a, b, c = _distinct_zipf(rng, vocab, 3)
        kinds.append(FILTER_BOOLEAN)
        pays.append([[a, b], [c]])  # (a AND b) OR c
    return kinds, pays


def make_config(name: str, n: Optional[int] = None, nq: Optional[int] = None,
                seed: int = 0) -> Workload:
    """Build one of the five workload shapes (optionally at a reduced size)."""
    if name == "c1":
        n = 20_000 if n is None else n
        nq = 100 if nq is None else nq
        rng = np.random.default_rng(seed)
        X, C = mixture(rng, n, 32, 16)
        labels = rng.integers(0, 8, size=n).astype(np.int32)
        loff = np.arange(n + 1, dtype=np.int64)
        rq = np.random.default_rng(seed + 1)
        Q, _ = mixture(rq, nq, 32, 16, centers=C)
        fl = rq.integers(0, 8, size=nq)
        F, pool = encode_filters([FILTER_LABEL] * nq, fl.tolist())
        return Workload("c1", X, Q, F, pool, None, loff, labels, 8, k=10, R=32, L=64,
                        meta=dict(clusters=16, thresholds="label{100%,0}"))
    if name == "c2":
        n = 1_000_000 if n is None else n
        nq = 10_000 if nq is None else nq
        rng = np.random.default_rng(seed)
        X, C = mixture(rng, n, 96, 256)
        scalar = rng.integers(0, RANGE_DOMAIN, size=n).astype(np.int32)
        rq = np.random.default_rng(seed + 1)
        Q, _ = mixture(rq, nq, 96, 256, centers=C)
        lo, hi = range_filters(rq, nq)
        F, pool = encode_filters([FILTER_RANGE] * nq, list(zip(lo.tolist(), hi.tolist())))
        return Workload("c2", X, Q, F, pool, scalar, None, None, 0, k=10, R=64, L=64,
                        meta=dict(clusters=256, thresholds="scalar{100%,1%,0}"))
    if name == "c3":
        n = 1_000_000 if n is None else n
        nq = 10_000 if nq is None else nq
        rng = np.random.default_rng(seed)
        X, C = mixture(rng, n, 128, 256)
        loff, lab = zipf_label_sets(np.random.default_rng(seed + 7), n, 1000, 1, 10)
        rq = np.random.default_rng(seed + 1)
        Q, _ = mixture(rq, nq, 128, 256, centers=C)
        kinds, pays = _subset_and_bool_queries(rq, nq // 2, nq - nq // 2, 1000)
        F, pool = encode_filters(kinds, pays)
        return Workload("c3", X, Q, F, pool, None, loff, lab, 1000, k=10, R=64, L=64,
                        meta=dict(clusters=256, thresholds="labels{100%,1%,0}"))
    if name == "c4":
        base = make_config("c1", n=n, nq=1, seed=seed)
        n = base.n
        nq = 10_000 if nq is None else nq
        r1 = np.random.default_rng(seed + 1)
        scalar = r1.integers(0, RANGE_DOMAIN, size=n).astype(np.int32)
        r2 = np.random.default_rng(seed + 2)
        extra = r2.integers(0, 3, size=n)
        sets = []
        for i in range(n):
            s = {int(base.lab[i])}
            while len(s) < 1 + extra[i]:
                s.add(int(r2.integers(0, 8)))
            sets.append(sorted(s))
        loff = np.zeros(n + 1, dtype=np.int64)
        loff[1:] = np.cumsum([len(s) for s in sets])
        lab = np.fromiter((v for s in sets for v in s), dtype=np.int32, count=int(loff[-1]))
        rq = np.random.default_rng(seed + 3)
        C = base.meta.get("centers")
        Q, _ = mixture(rq, nq, 32, 16, centers=_c1_centers(seed))
        t = rq.integers(0, 3, size=nq)
        lo, hi = range_filters(rq, nq)
        kinds, pays = [], []
        for i in range(nq):
            if t[i] == 0:
                kinds.append(FILTER_LABEL)
                pays.append(int(rq.integers(0, 8)))
            elif t[i] == 1:
                kinds.append(FILTER_RANGE)
                pays.append((int(lo[i]), int(hi[i])))
            else:
                m = int(rq.integers(1, 3))
                kinds.append(FILTER_SUBSET)
                pays.append(sorted(rq.choice(8, size=m, replace=False).tolist()))
        F, pool = encode_filters(kinds, pays)
        del C
        return Workload("c4", base.X, Q, F, pool, scalar, loff, lab, 8, k=10, R=32, L=64,
                        meta=dict(clusters=16, thresholds="scalar{100%,1%,0}+labels{1%,0}"))
    if name == "bool15":
        # general Boolean filters (the paper's synthetic Boolean workload,
        # App. D.2): every item holds a random assignment of 15 binary
        # variables (label i present with probability 1/2), every query a
        # random Boolean function of them whose pass rate is log-uniform in
        # one of four ranges (2^-4, 1), (2^-8, 2^-4), (2^-12, 2^-8), (0, 2^-12)
        n = 1_000_000 if n is None else n
        nq = 10_000 if nq is None else nq
        rng = np.random.default_rng(seed)
        X, C = mixture(rng, n, 96, 256)
        bits = rng.random((n, 15)) < 0.5
        loff = np.zeros(n + 1, dtype=np.int64)
        loff[1:] = np.cumsum(bits.sum(1))
        lab = np.nonzero(bits)[1].astype(np.int32)
        rq = np.random.default_rng(seed + 1)
        Q, _ = mixture(rq, nq, 96, 256, centers=C)
        kinds, pays = _table_queries(rq, nq)
        F, pool = encode_filters(kinds, pays)
        return Workload("bool15", X, Q, F, pool, None, loff, lab, 15, k=10, R=64, L=64,
                        meta=dict(clusters=256, thresholds="labels{100%,1%,0}"))
    if name == "c5":
        n = 10_000_000 if n is None else n
        nq = 10_000 if nq is None else nq
        rng = np.random.default_rng(seed)
        X, C = mixture(rng, n, 100, 1024)
        scalar = rng.integers(0, RANGE_DOMAIN, size=n).astype(np.int32)
        loff, lab = zipf_label_sets(np.random.default_rng(seed + 7), n, 1000, 1, 5)
        rq = np.random.default_rng(seed + 1)
        Q, _ = mixture(rq, nq, 100, 1024, centers=C)
        t = np.arange(nq) % 4
        rq.shuffle(t)
        lo, hi = range_filters(rq, nq)
        kinds, pays = [], []
        for i in range(nq):
            if t[i] == FILTER_LABEL:
                kinds.append(FILTER_LABEL)
                pays.append(_distinct_zipf(rq, 1000, 1)[0])
            elif t[i] == FILTER_RANGE:
                kinds.append(FILTER_RANGE)
                pays.append((int(lo[i]), int(hi[i])))
            elif t[i] == FILTER_SUBSET:
                kinds.append(FILTER_SUBSET)
                pays.append(sorted(_distinct_zipf(rq, 1000, int(rq.integers(1, 4)))))
            else:
                a, b, c = _distinct_zipf(rq, 1000, 3)
                kinds.append(FILTER_BOOLEAN)
                pays.append([[a, b], [c]])
        F, pool = encode_filters(kinds, pays)
        return Workload("c5", X, Q, F, pool, scalar, loff, lab, 1000, k=10, R=64, L=64,
                        meta=dict(clusters=1024, thresholds="scalar{100%,1%,0}+labels{1%,0}"))
    raise ValueError(f"unknown config {name}")


def _c1_centers(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 4.0, size=(16, 32))


_SHAPES = {"c1": (32, 16), "c2": (96, 256), "c3": (128, 256), "c4": (32, 16), "c5": (100, 1024),
           "bool15": (96, 256)}


def _table_queries(rq, nq: int):
    """Random Boolean functions of 15 variables (labels 0..14), query i with
    a pass rate log-uniform in range i % 4 of (2^-4, 1), (2^-8, 2^-4),
    (2^-12, 2^-8), (2^-15, 2^-12); at least one true assignment."""
    kinds, pays = [], []
    lo_exp = [(-4, 0), (-8, -4), (-12, -8), (-15, -12)]
    for i in range(nq):
        a, b = lo_exp[i % 4]
        rate = 2.0 ** rq.uniform(a, b)
        m = max(1, int(round(rate * 32768)))
        table = np.zeros(32768, dtype=bool)
        table[rq.choice(32768, size=m, replace=False)] = True
        kinds.append(FILTER_TABLE)
        pays.append((list(range(15)), table))
    return kinds, pays


def extra_queries(w: Workload, nq: int, qseed: int, seed: int = 0):
    """A further query set with the recipe of workload ``w`` (same mixture
    centres, different seed), e.g. for fitting the beam predictor.
    Returns (Q, F, pool)."""
    d, clusters = _SHAPES[w.name]
    centers = np.random.default_rng(seed).normal(0.0, 4.0, size=(clusters, d))
    rq = np.random.default_rng(qseed)
    Q, _ = mixture(rq, nq, d, clusters, centers=centers)
    if w.name == "c1":
        F, pool = encode_filters([FILTER_LABEL] * nq, rq.integers(0, 8, size=nq).tolist())
    elif w.name == "c2":
        lo, hi = range_filters(rq, nq)
        F, pool = encode_filters([FILTER_RANGE] * nq, list(zip(lo.tolist(), hi.tolist())))
    elif w.name == "c3":
        kinds, pays = _subset_and_bool_queries(rq, nq // 2, nq - nq // 2, 1000)
        F, pool = encode_filters(kinds, pays)
    elif w.name == "bool15":
        F, pool = encode_filters(*_table_queries(rq, nq))
    else:
        kinds, pays = [], []
        lo, hi = range_filters(rq, nq)
        vocab = w.vocab
        ntypes = 3 if w.name == "c4" else 4
        t = rq.integers(0, ntypes, size=nq)
        for i in range(nq):
            if t[i] == FILTER_LABEL:
                kinds.append(FILTER_LABEL)
                pays.append(int(rq.integers(0, 8)) if w.name == "c4" else _distinct_zipf(rq, vocab, 1)[0])
            elif t[i] == FILTER_RANGE:
                kinds.append(FILTER_RANGE)
                pays.append((int(lo[i]), int(hi[i])))
            elif t[i] == FILTER_SUBSET:
                kinds.append(FILTER_SUBSET)
                if w.name == "c4":
                    pays.append(sorted(rq.choice(8, size=int(rq.integers(1, 3)), replace=False).tolist()))
                else:
                    pays.append(sorted(_distinct_zipf(rq, vocab, int(rq.integers(1, 4)))))
            else:
                a, b, c = _distinct_zipf(rq, vocab, 3)
                kinds.append(FILTER_BOOLEAN)
                pays.append([[a, b], [c]])
        F, pool = encode_filters(kinds, pays)
    return Q, F, pool


def poisson_arrivals(rng: np.random.Generator, nq: int, qps: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream at rate ``qps``."""
    return np.cumsum(rng.exponential(1.0 / qps, size=nq))
