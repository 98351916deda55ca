"""Python binding of libjag (include/jag.h): argument marshalling only.

Every function here has the name of the C entry point it calls and passes
plain pointers through; all of the search runs in the library's HIP
kernels.  Device buffers are torch CUDA tensors (PyTorch provides device
memory and streams only).  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjag.so")

JAG_OK, JAG_EINVAL, JAG_ENOMEM, JAG_EDEVICE, JAG_EIO, JAG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STORE_F32, STORE_BF16, STORE_FP8_E4M3 = 0, 1, 2
LABEL, RANGE, SUBSET, BOOLEAN = 0, 1, 2, 3
ATTR_SCALAR, ATTR_LABELS, ATTR_LABELS_WEIGHTED = 0, 1, 2
FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, FILTER_BOOLEAN, FILTER_TABLE = 0, 1, 2, 3, 4
THRESHOLD_WEIGHT = 0x100  # flag on a threshold kind: Weight-JAG entry, quantile = weight multiplier
FILTER_RECORD_BYTES = 128
LADDER_MAX = 16
N_PARAMS = 5313


class JagError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"jag error {status}: {msg}")
        self.status = status


class jag_attrs(C.Structure):
    _fields_ = [("scalar", C.c_void_p), ("label_off", C.c_void_p), ("labels", C.c_void_p),
                ("vocab", C.c_int32)]


class jag_threshold(C.Structure):
    _fields_ = [("kind", C.c_int32), ("quantile", C.c_float)]


class jag_build_params(C.Structure):
    _fields_ = [("R", C.c_int32), ("L_build", C.c_int32), ("alpha", C.c_float),
                ("n_thr", C.c_int32), ("thr", C.POINTER(jag_threshold)), ("store", C.c_int32),
                ("keep_f32", C.c_int32), ("seed", C.c_uint64), ("n_threads", C.c_int32),
                ("max_batch", C.c_int32), ("progress", C.c_int32), ("device", C.c_int32),
                ("order", C.c_void_p), ("thresholds", C.c_void_p)]


class jag_search_params(C.Structure):
    _fields_ = [("L", C.c_int32), ("learned", C.c_int32), ("delta", C.c_float),
                ("rerank_mult", C.c_int32), ("max_hops", C.c_int32), ("stats", C.c_void_p),
                ("features", C.c_void_p), ("hash_log2", C.c_int32),
                ("single_pass", C.c_int32)]


class jag_index_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("R", C.c_int32), ("entry", C.c_int32),
                ("store", C.c_int32), ("has_f32", C.c_int32), ("has_scalar", C.c_int32),
                ("has_labels", C.c_int32), ("label_width", C.c_int32), ("vocab", C.c_int32),
                ("has_predictor", C.c_int32), ("device_bytes", C.c_int64)]


_lib = None


def lib():
    """Load libjag.so (built by paper_2602_10258_amd.build); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2602_10258_amd.build`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 under
        # the same soname.  Loaded first, it is the one libjag binds to;
        # loaded after libjag, a second HIP and HSA runtime would be mapped
        # beside the system's and PyTorch would find no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_uint64
        sig = {
            "jag_build": ([P, i64, i32, P, P, P], i32),
            "jag_build_graph": ([P, i64, i32, P, P, P, P], i32),
            "jag_build_from_graph": ([P, i64, i32, P, P, i32, i32, P, P], i32),
            "jag_save": ([P, C.c_char_p], i32),
            "jag_load": ([C.c_char_p, P], i32),
            "jag_free": ([P], None),
            "jag_info": ([P, P], i32),
            "jag_get_graph": ([P, P, P], i32),
            "jag_get_store": ([P, P, P], i32),
            "jag_encode_filters": ([P, P, i64, P, i64, P], i32),
            "jag_encoded_bytes": ([P, P, i64, P, i64, P], i32),
            "jag_encode_filters_sized": ([P, P, i64, P, i64, P, i64], i32),
            "jag_search_encoded": ([P, P, i64, P, i32, P, P, P, P, P], i32),
            "jag_search_encoded_noalloc": ([P, P, i64, P, i32, P, P, P, P, P], i32),
            "jag_search_batch": ([P, P, i64, P, P, i64, i32, P, P, P, P, P], i32),
            "jag_exact_knn": ([P, P, i64, P, i32, P, P, P, P], i32),
            "jag_set_predictor": ([P, P, i32, P, f32], i32),
            "jag_train_predictor": ([P, P, i64, P, i32, i32, f32, u64, P, P], i32),
            "jag_predictor_grad": ([P, P, i64, P, P, P, P], i32),
            "jag_gather_ceiling": ([P, i64, i32, i32, i32, i32, P, P], i32),
            "jag_last_error": ([], C.c_char_p),
            "jag_version": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return ["jag_build", "jag_build_graph", "jag_build_from_graph", "jag_save", "jag_load", "jag_free", "jag_info",
            "jag_get_graph", "jag_get_store", "jag_encode_filters", "jag_encoded_bytes",
            "jag_encode_filters_sized", "jag_search_encoded", "jag_search_encoded_noalloc",
            "jag_search_batch", "jag_exact_knn", "jag_set_predictor", "jag_train_predictor",
            "jag_predictor_grad", "jag_gather_ceiling", "jag_last_error", "jag_version", "jag_server_start",
            "jag_server_submit", "jag_server_poll", "jag_server_drain", "jag_server_stats_get",
            "jag_server_stop"]


def _check(st: int):
    if st != JAG_OK:
        raise JagError(st, lib().jag_last_error().decode())


def _np(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _attrs(scalar, label_off, labels, vocab):
    keep = (_np(scalar, np.int32), _np(label_off, np.int64), _np(labels, np.int32))
    a = jag_attrs(_ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), int(vocab))
    return a, keep


def _params(R, L_build, alpha, thresholds, store, keep_f32, seed, n_threads, max_batch, progress=False,
            device=False, order=None, thr_values=None):
    """jag_build_params and the buffers it points to (keep them alive with it)."""
    thr = (jag_threshold * max(1, len(thresholds)))(*[jag_threshold(int(k), float(q)) for k, q in thresholds])
    order = _np(order, np.int32)
    thr_values = _np(thr_values, np.float32)
    p = jag_build_params(int(R), int(L_build), float(alpha), len(thresholds),
                         C.cast(thr, C.POINTER(jag_threshold)), int(store), int(keep_f32),
                         int(seed), int(n_threads), int(max_batch), int(bool(progress)),
                         int(bool(device)), _ptr(order), _ptr(thr_values))
    return p, (thr, order, thr_values)


def _check_plan_inputs(n, nthr, order, thr_values):
    """The C ABI cannot see array lengths: check them here."""
    if order is not None and np.shape(order) != (n,):
        raise ValueError(f"order must have shape ({n},)")
    if thr_values is not None and np.shape(thr_values) != (n, nthr):
        raise ValueError(f"thr_values must have shape ({n}, {nthr})")


class Index:
    """Owning handle of a jag_index."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise ValueError("index already freed")
        return self._h

    def free(self):
        if self._h:
            lib().jag_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> jag_index_info:
        out = jag_index_info()
        _check(lib().jag_info(self.handle, C.byref(out)))
        return out


def jag_build(X, scalar=None, label_off=None, labels=None, vocab=0, R=32, L_build=0, alpha=1.2,
              thresholds: Sequence = ((ATTR_SCALAR, 1.0),), store=STORE_F32, keep_f32=False,
              seed=0, n_threads=0, max_batch=0, device=False, order=None, thr_values=None) -> Index:
    X = _np(X, np.float32)
    _check_plan_inputs(X.shape[0], len(thresholds), order, thr_values)
    a, keep = _attrs(scalar, label_off, labels, vocab)
    p, thr = _params(R, L_build, alpha, thresholds, store, keep_f32, seed, n_threads, max_batch,
                     False, device, order, thr_values)
    h = C.c_void_p()
    _check(lib().jag_build(_ptr(X), X.shape[0], X.shape[1], C.byref(a), C.byref(p), C.byref(h)))
    return Index(h)


def jag_build_graph(X, scalar=None, label_off=None, labels=None, vocab=0, R=32, L_build=0,
                    alpha=1.2, thresholds: Sequence = ((ATTR_SCALAR, 1.0),), seed=0, n_threads=0,
                    max_batch=0, progress=False, device=False, order=None, thr_values=None):
    """Threshold-/Weight-JAG construction on host threads (device=False) or on
    the current GPU (device=True, the same graph); returns (adj int32[n, R], entry).
    order: optional insertion order (order[0] becomes the entry vertex);
    thr_values: optional float32 [n, len(thresholds)] per-point t / w values."""
    X = _np(X, np.float32)
    _check_plan_inputs(X.shape[0], len(thresholds), order, thr_values)
    a, keep = _attrs(scalar, label_off, labels, vocab)
    p, thr = _params(R, L_build, alpha, thresholds, STORE_F32, 0, seed, n_threads, max_batch, progress,
                     device, order, thr_values)
    adj = np.empty((X.shape[0], R), dtype=np.int32)
    e = C.c_int32()
    _check(lib().jag_build_graph(_ptr(X), X.shape[0], X.shape[1], C.byref(a), C.byref(p), _ptr(adj),
                                 C.byref(e)))
    return adj, int(e.value)


def jag_build_from_graph(X, adj, entry, scalar=None, label_off=None, labels=None, vocab=0,
                         store=STORE_F32, keep_f32=False) -> Index:
    X = _np(X, np.float32)
    adj = _np(adj, np.int32)
    a, keep = _attrs(scalar, label_off, labels, vocab)
    p, thr = _params(1, 0, 1.2, [], store, keep_f32, 0, 0, 0)
    h = C.c_void_p()
    _check(lib().jag_build_from_graph(_ptr(X), X.shape[0], X.shape[1], C.byref(a), _ptr(adj),
                                      adj.shape[1], int(entry), C.byref(p), C.byref(h)))
    return Index(h)


def jag_save(idx: Index, path: str):
    _check(lib().jag_save(idx.handle, path.encode()))


def jag_load(path: str) -> Index:
    h = C.c_void_p()
    _check(lib().jag_load(path.encode(), C.byref(h)))
    return Index(h)


def jag_free(idx: Index):
    idx.free()


def jag_get_graph(idx: Index):
    info = idx.info()
    adj = np.empty((info.n, info.R), dtype=np.int32)
    e = C.c_int32()
    _check(lib().jag_get_graph(idx.handle, _ptr(adj), C.byref(e)))
    return adj, int(e.value)


def jag_get_store(idx: Index):
    info = idx.info()
    dt = {STORE_F32: np.float32, STORE_BF16: np.uint16, STORE_FP8_E4M3: np.uint8}[info.store]
    rows = np.empty((info.n, info.d), dtype=dt)
    scales = np.empty(info.n, dtype=np.float32) if info.store == STORE_FP8_E4M3 else None
    _check(lib().jag_get_store(idx.handle, _ptr(rows), _ptr(scales)))
    return rows, scales


def jag_encode_filters(idx: Index, F, pool) -> np.ndarray:
    """Encode int32 filter rows (type, label, lo, hi, off, len) into host records:
    uint8 [nq, FILTER_RECORD_BYTES], or, when the batch holds TABLE filters, one
    flat uint8 buffer of the records followed by their distance tables
    (jag_encode_filters_sized)."""
    F = _np(F, np.int32)
    pool = _np(pool, np.int32)
    nq = F.shape[0]
    if nq and np.any(F[:, 0] == FILTER_TABLE):
        need = C.c_int64()
        _check(lib().jag_encoded_bytes(idx.handle, _ptr(F), nq, _ptr(pool), pool.size, C.byref(need)))
        out = np.empty(need.value, dtype=np.uint8)
        _check(lib().jag_encode_filters_sized(idx.handle, _ptr(F), nq, _ptr(pool), pool.size, _ptr(out),
                                              need.value))
        return out
    out = np.empty((nq, FILTER_RECORD_BYTES), dtype=np.uint8)
    _check(lib().jag_encode_filters(idx.handle, _ptr(F), nq, _ptr(pool), pool.size, _ptr(out)))
    return out


@dataclass
class SearchParams:
    L: int = 64
    learned: int = 0
    delta: float = 0.0
    rerank_mult: int = 0
    max_hops: int = 0
    stats: Optional[object] = None      # torch int32 [nq, 4] on the device
    features: Optional[object] = None   # torch float32 [nq, 16] on the device
    hash_log2: int = 0
    single_pass: int = 0

    def c(self) -> jag_search_params:
        return jag_search_params(int(self.L), int(self.learned), float(self.delta),
                                 int(self.rerank_mult), int(self.max_hops), _ptr(self.stats),
                                 _ptr(self.features), int(self.hash_log2),
                                 int(self.single_pass))


def jag_search_encoded(idx: Index, Q, records, k: int, params: SearchParams, ids, dists, count,
                       stream=None):
    """Q, records (uint8 [nq,128]), ids, dists, count: torch tensors on the device."""
    sp = params.c()
    _check(lib().jag_search_encoded(idx.handle, _ptr(Q), Q.shape[0], _ptr(records), int(k),
                                    C.byref(sp), _ptr(ids), _ptr(dists), _ptr(count),
                                    _stream(stream)))


def jag_search_encoded_noalloc(idx: Index, Q, records, k: int, params: SearchParams, ids, dists, count,
                               stream=None):
    """jag_search_encoded with its scratch in the library's fixed device array
    (no device allocation; calls overlapping on one GPU race)."""
    sp = params.c()
    _check(lib().jag_search_encoded_noalloc(idx.handle, _ptr(Q), Q.shape[0], _ptr(records), int(k),
                                            C.byref(sp), _ptr(ids), _ptr(dists), _ptr(count),
                                            _stream(stream)))


def jag_search_batch(idx: Index, Q, F, pool, k: int, params: SearchParams, ids, dists, count,
                     stream=None):
    F = _np(F, np.int32)
    pool = _np(pool, np.int32)
    sp = params.c()
    _check(lib().jag_search_batch(idx.handle, _ptr(Q), Q.shape[0], _ptr(F), _ptr(pool), pool.size,
                                  int(k), C.byref(sp), _ptr(ids), _ptr(dists), _ptr(count),
                                  _stream(stream)))


def jag_exact_knn(idx: Index, Q, records, k: int, ids, dists, count, stream=None):
    _check(lib().jag_exact_knn(idx.handle, _ptr(Q), Q.shape[0], _ptr(records), int(k), _ptr(ids),
                               _ptr(dists), _ptr(count), _stream(stream)))


def jag_gather_ceiling(buffer, row_bytes: int, waves: int, iters: int, reps: int = 5, stream=None) -> float:
    """Random row-gather throughput (GB/s) over a device buffer (torch tensor)."""
    gbs = C.c_double()
    _check(lib().jag_gather_ceiling(_ptr(buffer), buffer.numel() * buffer.element_size(), int(row_bytes),
                                    int(waves), int(iters), int(reps), _stream(stream), C.byref(gbs)))
    return float(gbs.value)


def jag_set_predictor(idx: Index, params, ladder, rho: float):
    params = _np(params, np.float32)
    ladder = _np(ladder, np.int32)
    _check(lib().jag_set_predictor(idx.handle, _ptr(params), ladder.size, _ptr(ladder), float(rho)))


def jag_train_predictor(features, targets, params, epochs: int, batch: int, lr: float,
                        seed: int = 0, stream=None):
    """features/targets: torch device tensors; params: host float32[5313] (updated copy returned)."""
    p = np.array(params, dtype=np.float32, copy=True)
    loss = np.empty(epochs, dtype=np.float32)
    _check(lib().jag_train_predictor(_ptr(features), _ptr(targets), features.shape[0], _ptr(p),
                                     int(epochs), int(batch), float(lr), int(seed), _ptr(loss),
                                     _stream(stream)))
    return p, loss


def jag_predictor_grad(features, targets, params, stream=None):
    p = _np(params, np.float32)
    g = np.empty(N_PARAMS, dtype=np.float32)
    loss = np.empty(1, dtype=np.float32)
    _check(lib().jag_predictor_grad(_ptr(features), _ptr(targets), features.shape[0], _ptr(p),
                                    _ptr(loss), _ptr(g), _stream(stream)))
    return float(loss[0]), g


# ---------------------------------------------------------------- serving

class jag_server_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("search", jag_search_params), ("max_batch", C.c_int32),
                ("n_streams", C.c_int32), ("max_wait_us", C.c_int32), ("max_inflight", C.c_int64),
                ("queue_capacity", C.c_int64), ("hbm_budget_bytes", C.c_int64),
                ("slot_admission", C.c_int32), ("reserved", C.c_int32)]


class jag_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("max_inflight_seen", C.c_int64), ("resident_capacity", C.c_int64),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("mean_us", C.c_double),
                ("max_us", C.c_double), ("qps", C.c_double), ("mean_batch", C.c_double),
                ("device_bytes", C.c_int64)]


JAG_EBUSY, JAG_EAGAIN = -6, 1
_SERVER_SIG = {
    "jag_server_start": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int32),
    "jag_server_submit": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                           C.c_void_p], C.c_int32),
    "jag_server_poll": ([C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                        C.c_int32),
    "jag_server_drain": ([C.c_void_p], C.c_int32),
    "jag_server_stats_get": ([C.c_void_p, C.c_void_p], C.c_int32),
    "jag_server_stop": ([C.c_void_p], None),
}


def _server_lib():
    L = lib()
    if not getattr(L, "_server_sig_set", False):
        for name, (args, res) in _SERVER_SIG.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        L._server_sig_set = True
    return L


class Server:
    """Owning handle of a jag_server (keeps its index alive)."""

    def __init__(self, handle, idx: Index, k: int):
        self._h, self.idx, self.k = handle, idx, k

    def stop(self):
        if self._h:
            _server_lib().jag_server_stop(self._h)
            self._h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def jag_server_start(idx: Index, k: int, search: SearchParams, max_batch: int = 1024,
                     n_streams: int = 4, max_wait_us: int = 200, max_inflight: int = 0,
                     queue_capacity: int = 1 << 22, hbm_budget_bytes: int = 0,
                     slot_admission: bool = False) -> Server:
    p = jag_server_params(int(k), search.c(), int(max_batch), int(n_streams), int(max_wait_us),
                          int(max_inflight), int(queue_capacity), int(hbm_budget_bytes),
                          int(bool(slot_admission)), 0)
    h = C.c_void_p()
    _check(_server_lib().jag_server_start(idx.handle, C.byref(p), C.byref(h)))
    return Server(h, idx, k)


def jag_server_submit(s: Server, Q, F, pool) -> np.ndarray:
    Q = _np(Q, np.float32)
    F = _np(F, np.int32)
    pool = _np(pool, np.int32)
    n = F.shape[0]
    t = np.empty(n, dtype=np.uint64)
    _check(_server_lib().jag_server_submit(s._h, _ptr(Q), _ptr(F), n, _ptr(pool), pool.size, _ptr(t)))
    return t


def jag_server_poll(s: Server, ticket: int):
    """(ids, dists, count, latency_us) when done, None while pending."""
    ids = np.empty(s.k, dtype=np.int32)
    d = np.empty(s.k, dtype=np.float32)
    c = C.c_int32()
    lat = C.c_double()
    st = _server_lib().jag_server_poll(s._h, int(ticket), _ptr(ids), _ptr(d), C.byref(c), C.byref(lat))
    if st == JAG_EAGAIN:
        return None
    _check(st)
    return ids, d, int(c.value), float(lat.value)


def jag_server_drain(s: Server):
    _check(_server_lib().jag_server_drain(s._h))


def jag_server_stats_get(s: Server) -> dict:
    o = jag_server_stats()
    _check(_server_lib().jag_server_stats_get(s._h, C.byref(o)))
    return {f: getattr(o, f) for f, _ in jag_server_stats._fields_}


def jag_server_stop(s: Server):
    s.stop()
