"""ctypes wrapper around the plain CPU reference (``jag_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the CPU
baseline leg of the benchmark use this module.  The product library never
imports it.  See ``jag_oracle.c`` for what each routine computes and which
part of the paper it follows.

Parity status: every routine here is pinned by ``tests/test_oracle_*.py``;
the graph builder by graphs worked out by hand on two five-point worlds
(``tests/golden/build_line_worlds.txt``) besides structural invariants and
recall.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jag_oracle.c")
_LIB = os.path.join(_HERE, "libjag_oracle.so")

KIND_SCALAR, KIND_LABELS, KIND_LABELS_WEIGHTED = 0, 1, 2
WEIGHT_ENTRY = 0x100  # flag on a build entry kind: Weight-JAG comparator, quantile = weight multiplier
N_PARAMS = 5313
LADDER = np.array([16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512], dtype=np.int32)


def build_library(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build_library()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, f64, f32, u64 = C.c_int64, C.c_int32, C.c_double, C.c_float, C.c_uint64
        L.or_search.argtypes = [i64, i32, P, P, i32, i32, P, P, P, i64, P, P, P, i32, i32, P, i32,
                                P, f32, f32, i32, P, P, i32, P, P, P, P, P, P, P, P, P, P]
        L.or_search.restype = C.c_int
        L.or_bruteforce.argtypes = [i64, i32, P, P, P, P, i64, P, P, P, i32, i32, P, P, P]
        L.or_bruteforce.restype = C.c_int
        L.or_dist_f_pairs.argtypes = [i64, P, P, P, i64, P, P, P, P, P]
        L.or_dist_f_pairs.restype = None
        L.or_dist_a_pairs.argtypes = [i64, P, P, P, i32, i64, P, P, f64, P]
        L.or_dist_a_pairs.restype = None
        L.or_build.argtypes = [i64, i32, P, P, P, P, i32, i32, f64, i32, P, P, u64, P, P, P, P, P]
        L.or_build.restype = i32
        L.or_prune.argtypes = [i64, i32, P, P, P, P, i32, f64, i32, P, P, i32, P, i32, P]
        L.or_prune.restype = i32
        L.or_bf16_encode_array.argtypes = [i64, P, P]
        L.or_bf16_encode_array.restype = None
        L.or_e4m3_value.argtypes = [C.c_uint8]
        L.or_e4m3_value.restype = f64
        L.or_e4m3_encode.argtypes = [f32]
        L.or_e4m3_encode.restype = C.c_uint8
        L.or_fp8_encode_rows.argtypes = [i64, i32, P, P, P]
        L.or_fp8_encode_rows.restype = None
        L.or_fp8_decode_rows.argtypes = [i64, i32, P, P, P]
        L.or_fp8_decode_rows.restype = None
        L.or_selectivity.argtypes = [i64, P, P, P, i64, P, P, P]
        L.or_selectivity.restype = None
        L.or_mlp_forward.argtypes = [P, i64, P, P]
        L.or_mlp_forward.restype = None
        L.or_mlp_loss_grad.argtypes = [P, i64, P, P, P, P]
        L.or_mlp_loss_grad.restype = f64
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Attrs:
    """Per-item attributes: an int32 scalar and/or CSR label sets (rows sorted)."""
    n: int
    scalar: Optional[np.ndarray] = None
    loff: Optional[np.ndarray] = None
    lab: Optional[np.ndarray] = None

    def arrays(self):
        return (_c(self.scalar, np.int32), _c(self.loff, np.int64), _c(self.lab, np.int32))


def attrs_of(w) -> Attrs:
    return Attrs(w.n, w.scalar, w.loff, w.lab)


def dist_f(attrs: Attrs, items, F, fidx, pool) -> np.ndarray:
    """dist_F(a_item, filter) for pairs (items[j], F[fidx[j]]) -- Section 3.1."""
    s, lo, lb = attrs.arrays()
    items = _c(items, np.int64)
    F = _c(F, np.int32)
    fidx = _c(fidx, np.int32)
    pool = _c(pool, np.int32)
    out = np.empty(len(items), dtype=np.float64)
    lib().or_dist_f_pairs(attrs.n, _p(s), _p(lo), _p(lb), len(items), _p(items), _p(F),
                          _p(fidx), _p(pool), _p(out))
    return out


def selectivity(attrs: Attrs, F, pool) -> np.ndarray:
    """Selectivity estimate per filter: exact fraction for label and range
    filters; for subset, DNF and table filters the probability of passing
    when labels are held independently with their observed frequencies."""
    s, lo, lb = attrs.arrays()
    F = _c(F, np.int32)
    pool = _c(pool, np.int32)
    out = np.empty(F.shape[0], dtype=np.float64)
    lib().or_selectivity(attrs.n, _p(s), _p(lo), _p(lb), F.shape[0], _p(F), _p(pool), _p(out))
    return out


def sel_feature(sel) -> np.ndarray:
    """The predictor's selectivity feature log2(max(s, 1e-9)) / 16, as float32."""
    sel = np.asarray(sel, dtype=np.float64)
    return (np.log2(np.maximum(sel, 1e-9)) / 16.0).astype(np.float32)


def dist_a(attrs: Attrs, kind: int, i1, i2, t: float = 0.0) -> np.ndarray:
    """Capped attribute distance max(dist_A - t, 0) -- Section 3.2."""
    s, lo, lb = attrs.arrays()
    i1 = _c(i1, np.int64)
    i2 = _c(i2, np.int64)
    out = np.empty(len(i1), dtype=np.float64)
    lib().or_dist_a_pairs(attrs.n, _p(s), _p(lo), _p(lb), kind, len(i1), _p(i1), _p(i2),
                          float(t), _p(out))
    return out


def _out_i32(a: Optional[np.ndarray], n: int):
    if a is None:
        return None
    if a.dtype != np.int32 or a.shape != (n,) or not a.flags.c_contiguous:
        raise ValueError("order_out must be a contiguous int32 array of n entries")
    return a


def build(X, attrs: Attrs, R: int, L_build: int, alpha: float, kinds, quantiles,
          seed: int = 0, order_out: Optional[np.ndarray] = None, order=None, thresholds=None):
    """Sequential Threshold-JAG build (Algorithms 3-4).  Returns (adj, entry, thr);
    the insertion order goes to order_out (int32 [n]) when given.  ``order``
    (a permutation starting with the entry vertex) and ``thresholds``
    (float64 [n][|T|]) replace the seeded order and the sampled thresholds."""
    X = _c(X, np.float32)
    n, d = X.shape
    s, lo, lb = attrs.arrays()
    kinds = _c(kinds, np.int32)
    quant = _c(quantiles, np.float64)
    order = _c(order, np.int32)
    thr_in = _c(thresholds, np.float64)
    if order is not None and order.shape != (n,):
        raise ValueError("order must hold n entries")
    if thr_in is not None and thr_in.shape != (n, len(kinds)):
        raise ValueError("thresholds must be [n][len(kinds)]")
    adj = np.empty((n, R), dtype=np.int32)
    thr = np.empty((n, len(kinds)), dtype=np.float64)
    entry = lib().or_build(n, d, _p(X), _p(s), _p(lo), _p(lb), R, L_build, float(alpha),
                           len(kinds), _p(kinds), _p(quant), seed, _p(adj), _p(thr),
                           _p(_out_i32(order_out, n)), _p(order), _p(thr_in))
    if entry < 0:
        raise ValueError("order is not a permutation starting with the entry vertex")
    return adj, int(entry), thr


def prune(X, attrs: Attrs, R: int, alpha: float, kinds, thr, p: int, cand):
    """JointRobustPrune(G, p, V=cand, R, alpha, T) with explicit thresholds thr[n][|T|]."""
    X = _c(X, np.float32)
    n, d = X.shape
    s, lo, lb = attrs.arrays()
    kinds = _c(kinds, np.int32)
    thr = _c(thr, np.float64)
    cand = _c(cand, np.int32)
    out = np.empty(R, dtype=np.int32)
    m = lib().or_prune(n, d, _p(X), _p(s), _p(lo), _p(lb), R, float(alpha), len(kinds), _p(kinds),
                       _p(thr), p, _p(cand), len(cand), _p(out))
    return out[:m].tolist()


@dataclass
class SearchResult:
    ids: np.ndarray
    d2: np.ndarray
    count: np.ndarray
    hops: np.ndarray
    dc: np.ndarray
    margin: np.ndarray
    y: np.ndarray
    lhat: np.ndarray
    feat: np.ndarray  # [nq][16] predictor features (NaN without a predictor)


def search(base, adj, entry, attrs: Attrs, Q, F, pool, L: int, k: int, rerank=None,
           rerank_mult: int = 4, learned=None, delta: float = 0.0, rho: float = 1e9,
           ladder=LADDER, sel_feature=None, nthreads: int = 1, contract=None) -> SearchResult:
    """Query (Algorithm 2 over Algorithm 1) for a batch of filtered queries.

    ``base`` holds the vectors the search ranks by (FP32, or the exact
    decoding of a BF16/FP8 store); ``rerank`` optionally holds FP32 vectors
    used to rescore the best ``rerank_mult * k`` entries of the final list.
    ``learned`` is a float32[5313] parameter vector enabling the beam
    predictor.  ``contract`` = (G, EPC, CH) of the ranking vectors followed
    by those of the rescoring vectors selects FP32 distances in that lane
    order instead of FP64 (see ``sqdist_contract`` in the C source).
    """
    base = _c(base, np.float32)
    n, d = base.shape
    adj = _c(adj, np.int32)
    R = adj.shape[1]
    s, lo, lb = attrs.arrays()
    Q = _c(Q, np.float32)
    F = _c(F, np.int32)
    pool = _c(pool, np.int32)
    nq = Q.shape[0]
    rerank = _c(rerank, np.float32)
    learned = _c(learned, np.float32)
    ladder = _c(ladder, np.int32)
    self_ = _c(sel_feature, np.float32)
    ids = np.empty((nq, k), dtype=np.int32)
    d2 = np.empty((nq, k), dtype=np.float64)
    count = np.empty(nq, dtype=np.int32)
    hops = np.empty(nq, dtype=np.int32)
    dc = np.empty(nq, dtype=np.int32)
    margin = np.empty(nq, dtype=np.float64)
    y = np.empty(nq, dtype=np.float64)
    lhat = np.empty(nq, dtype=np.int32)
    feat = np.full((nq, 16), np.nan, dtype=np.float64)
    con = None if contract is None else np.ascontiguousarray(contract, dtype=np.int32)
    if con is not None and con.shape != (6,):
        raise ValueError("contract holds six integers")
    lib().or_search(n, d, _p(base), _p(adj), R, entry, _p(s), _p(lo), _p(lb), nq, _p(Q), _p(F),
                    _p(pool), L, k, _p(rerank), rerank_mult, _p(learned), float(delta),
                    float(rho), len(ladder), _p(ladder), _p(self_), nthreads, _p(ids), _p(d2),
                    _p(count), _p(hops), _p(dc), _p(margin), _p(y), _p(lhat), _p(feat), _p(con))
    return SearchResult(ids, d2, count, hops, dc, margin, y, lhat, feat)


def bruteforce(X, attrs: Attrs, Q, F, pool, k: int, nthreads: int = 1):
    """Exact filtered k-NN in FP64 (Pre-Filtering).  Returns (ids, d2, nvalid)."""
    X = _c(X, np.float32)
    n, d = X.shape
    s, lo, lb = attrs.arrays()
    Q = _c(Q, np.float32)
    F = _c(F, np.int32)
    pool = _c(pool, np.int32)
    nq = Q.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    d2 = np.empty((nq, k), dtype=np.float64)
    nvalid = np.empty(nq, dtype=np.int64)
    lib().or_bruteforce(n, d, _p(X), _p(s), _p(lo), _p(lb), nq, _p(Q), _p(F), _p(pool), k,
                        nthreads, _p(ids), _p(d2), _p(nvalid))
    return ids, d2, nvalid


def recall_at_k(ids, gt_ids, gt_d2, nvalid, k: int, X=None, Q=None) -> np.ndarray:
    """Per-query recall@k against the exact answer.

    Denominator min(k, #valid); queries with no valid item get NaN.  With
    X and Q given, a returned id also counts as a hit when its FP64 distance
    is no larger than the k-th exact distance (distance ties).
    """
    nq = ids.shape[0]
    out = np.full(nq, np.nan)
    for q in range(nq):
        den = min(k, int(nvalid[q]))
        if den == 0:
            continue
        gt = set(int(v) for v in gt_ids[q, :den])
        hits = 0
        kth = gt_d2[q, den - 1]
        for v in ids[q, :k]:
            v = int(v)
            if v < 0:
                continue
            if v in gt:
                hits += 1
            elif X is not None:
                dv = float(np.sum((X[v].astype(np.float64) - Q[q].astype(np.float64)) ** 2))
                if dv <= kth:
                    hits += 1
        out[q] = min(1.0, hits / den)
    return out


def bf16_encode(x) -> np.ndarray:
    x = _c(x, np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    lib().or_bf16_encode_array(x.size, _p(x), _p(out))
    return out


def bf16_decode(h) -> np.ndarray:
    h = np.asarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def e4m3_value(code: int) -> float:
    return lib().or_e4m3_value(code)


def e4m3_encode(y: float) -> int:
    return lib().or_e4m3_encode(float(y))


def fp8_encode_rows(X):
    X = _c(X, np.float32)
    n, d = X.shape
    codes = np.empty((n, d), dtype=np.uint8)
    scales = np.empty(n, dtype=np.float32)
    lib().or_fp8_encode_rows(n, d, _p(X), _p(codes), _p(scales))
    return codes, scales


def fp8_decode_rows(codes, scales):
    codes = _c(codes, np.uint8)
    scales = _c(scales, np.float32)
    n, d = codes.shape
    X = np.empty((n, d), dtype=np.float32)
    lib().or_fp8_decode_rows(n, d, _p(codes), _p(scales), _p(X))
    return X


def mlp_forward(params, X) -> np.ndarray:
    """Network output of the learned search's forward pass (FP32 parameters, FP64 sums)."""
    P = _c(params, np.float32)
    X = _c(X, np.float64)
    Y = np.empty(X.shape[0], dtype=np.float64)
    lib().or_mlp_forward(_p(P), X.shape[0], _p(X), _p(Y))
    return Y


def mlp_loss_grad(params, X, T):
    """FP64 loss (mean squared error) and gradient of the 16-64-64-1 network."""
    P = _c(params, np.float64)
    X = _c(X, np.float64)
    T = _c(T, np.float64)
    B = X.shape[0]
    G = np.empty(N_PARAMS, dtype=np.float64)
    Y = np.empty(B, dtype=np.float64)
    loss = lib().or_mlp_loss_grad(_p(P), B, _p(X), _p(T), _p(G), _p(Y))
    return loss, G, Y
