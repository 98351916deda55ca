"""Helpers for comparing the GPU search with the oracle (not a test module).

Trajectory tolerance.  The GPU sums squared differences in FP32: each lane
of a G-lane group accumulates m = (chunks x elements per chunk) terms with
fused multiply-adds, then the group adds its partial sums in log2(G)
butterfly steps.  With u = 2^-24, the rounding of q - x costs at most 2u per
term and every accumulation step at most u, so the relative error of one
distance is below eps = (m + 2 + log2 G) u.  Two keys whose exact relative
gap exceeds 2 eps are therefore ordered the same way by the GPU and by the
FP64 oracle.  The oracle reports, per query, the smallest relative gap of
any pair of keys whose order steered its search (selection, the l_s cut,
the rerank cut and the output order); every query whose margin is at least
tau = 2.02 eps must give identical ids.  tau stays below the 1e-5 relative
tie tolerance of the benchmark spec.
"""
from __future__ import annotations

import math

import numpy as np

U = 2.0 ** -24


def _layout(raw: int) -> tuple[int, int]:
    """(row stride, lanes per row) of the GPU's layout for rows of `raw` bytes:
    64-byte padding, then 4 lanes up to 384 bytes, 8 up to 512, 16 beyond, and
    padding to a multiple of 16 bytes per lane."""
    stride = (raw + 63) // 64 * 64
    G = 4 if stride <= 384 else 8 if stride <= 512 else 16
    return (stride + 16 * G - 1) // (16 * G) * (16 * G), G


def row_terms(store: int, d: int) -> tuple[int, int]:
    """(terms per lane, lanes per row) of the GPU distance for a store and dimension."""
    eb = {0: 4, 1: 2, 2: 1}[store]
    stride, G = _layout(eb * d + (4 if store == 2 else 0))
    ch = stride // (16 * G)
    epc = 16 // eb
    return ch * epc, G


def lane_order(store: int, d: int) -> list[int]:
    """The oracle's contract-mode order for the GPU's row layout: (G lanes,
    elements per 16-byte chunk, chunks per lane) of the search store, then
    of the FP32 rows the rerank reads.  The GPU splits those over lanes as
    it splits the store's rows (the same triple) when a lane's share is at
    most 32 elements, else four lanes take the 16-byte pieces of the
    64-byte-padded FP32 rows."""
    eb = {0: 4, 1: 2, 2: 1}[store]
    stride, G = _layout(eb * d + (4 if store == 2 else 0))
    out = [G, 16 // eb, stride // (16 * G)]
    if out[1] * out[2] <= 32:
        return out + out
    return out + [4, 4, _layout(4 * d)[0] // 64]


def compare_strict(gpu_ids, gpu_d2, gpu_cnt, orc, what=""):
    """Contract-mode oracle: every query's ids, count and FP32 distances equal."""
    bad = [q for q in range(gpu_ids.shape[0])
           if int(gpu_cnt[q]) != int(orc.count[q]) or not np.array_equal(gpu_ids[q], orc.ids[q])
           or not np.array_equal(gpu_d2[q, :gpu_cnt[q]].astype(np.float64), orc.d2[q, :gpu_cnt[q]])]
    assert not bad, f"{what}: {len(bad)} of {gpu_ids.shape[0]} queries differ, e.g. q={bad[0]} " \
                    f"gpu={gpu_ids[bad[0]].tolist()} oracle={orc.ids[bad[0]].tolist()}"


def tau_for(store: int, d: int, rerank_d: int | None = None) -> float:
    """tau for a search over `store` rows of d elements; with rerank_d, also
    for the FP32 rescoring (rows split as lane_order says)."""
    m, G = row_terms(store, d)
    eps = (m + 2 + math.log2(G)) * U
    if rerank_d is not None:
        m2, G2 = row_terms(store, rerank_d)
        if m2 > 32:  # the four-lane layout of wide rows
            m2, G2 = _layout(4 * rerank_d)[0] // 16, 4
        eps = max(eps, (m2 + 2 + math.log2(G2)) * U)
    tau = 2.02 * eps
    assert tau < 1e-5
    return tau


def compare(gpu_ids, gpu_d2, gpu_cnt, orc, tau, valid_fn=None, what=""):
    """Assert GPU == oracle on every query whose oracle margin >= tau.

    Returns (n_checked_exactly, n_flagged, n_flagged_differing).  Flagged
    queries (margin < tau) must still return valid, distinct ids in
    increasing distance order.
    """
    nq = gpu_ids.shape[0]
    exact = orc.margin >= tau
    bad = []
    flagged_diff = 0
    for q in range(nq):
        c = int(gpu_cnt[q])
        ids = gpu_ids[q]
        if exact[q]:
            if c != int(orc.count[q]) or not np.array_equal(ids, orc.ids[q]):
                bad.append(q)
                continue
            if c:
                rel = np.abs(gpu_d2[q, :c].astype(np.float64) - orc.d2[q, :c]) / np.maximum(orc.d2[q, :c], 1e-30)
                if rel.max() > 1e-5:
                    bad.append(q)
        else:
            if c != int(orc.count[q]) or not np.array_equal(ids, orc.ids[q]):
                flagged_diff += 1
            got = ids[:c]
            assert len(set(got.tolist())) == c, (what, q)
            assert np.all(ids[c:] == -1), (what, q)
            assert np.all(np.diff(gpu_d2[q, :c]) >= 0), (what, q)
            if valid_fn is not None and c:
                assert valid_fn(q, got), (what, q, got)
    assert not bad, f"{what}: {len(bad)} queries differ with margin >= {tau:.2e}: {bad[:10]}; " \
                    f"e.g. q={bad[0]} gpu={gpu_ids[bad[0]].tolist()} oracle={orc.ids[bad[0]].tolist()} " \
                    f"margin={orc.margin[bad[0]]:.3e}"
    return int(exact.sum()), int((~exact).sum()), flagged_diff
