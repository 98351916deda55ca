"""Fitting the learned beam-width predictor (not part of the paper).

Pipeline, all on the GPU through the C ABI:
  1. exact answers of the training queries (jag_exact_knn, Pre-Filtering);
  2. one traced search per ladder width L (learned == 2): the predictor
     features after four expansions, and the answer at L;
  3. target of a query = the smallest ladder index whose answer reaches
     recall@k >= 0.95 (for k = 10 that is every exact neighbour found); a
     query that reaches it nowhere on the ladder gets the widest index, or
     the smallest index at which its recall peaks;
  4. minibatch Adam on the GPU (jag_train_predictor), then jag_set_predictor
     with a hop cap rho = the 99th percentile of expansions / L at the target.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import jag

# beams the predictor chooses from; the widest equals the library's warm-up
# list width (64), so learned search needs no more LDS than fixed L = 64.
# Capping at 64 measured better at recall 0.95 on the range workload than a
# ladder to 128 (the clipped target is easier to fit; the queries that need
# more are the ones a 0.95 operating point gives up on anyway).
LADDER = np.array([10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64], dtype=np.int32)


@dataclass
class FitReport:
    n_train: int
    epochs: int
    loss_first: float
    loss_last: float
    rho: float
    target_hist: list
    unreachable: int


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation of the 16-64-64-1 network; output bias = mid-ladder."""
    rng = np.random.default_rng(seed)
    P = np.zeros(jag.N_PARAMS, dtype=np.float32)
    P[:1024] = rng.normal(0, np.sqrt(2.0 / 16), 1024)
    P[1088:5184] = rng.normal(0, np.sqrt(2.0 / 64), 4096)
    P[5248:5312] = rng.normal(0, np.sqrt(1.0 / 64), 64)
    P[5312] = len(LADDER) / 2
    return P


def _device_batch(idx, Q, F, pool):
    import torch
    rec = torch.from_numpy(jag.jag_encode_filters(idx, F, pool)).cuda()
    Qd = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).cuda()
    return Qd, rec


def traces(idx, Qd, rec, k: int, ladder=LADDER, rerank_mult: int = 0):
    """Features (nq x 16), per-ladder answers (nl x nq x k) and expansions (nl x nq)."""
    import torch
    nq = Qd.shape[0]
    feats = torch.zeros((nq, 16), dtype=torch.float32, device="cuda")
    stats = torch.zeros((nq, 4), dtype=torch.int32, device="cuda")
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    cnt = torch.empty((nq,), dtype=torch.int32, device="cuda")
    all_ids, hops = [], []
    for L in ladder:
        sp = jag.SearchParams(L=int(max(L, k)), learned=2, stats=stats, features=feats,
                              rerank_mult=rerank_mult)
        jag.jag_search_encoded(idx, Qd, rec, k, sp, ids, d2, cnt)
        torch.cuda.synchronize()
        all_ids.append(ids.cpu().numpy().copy())
        hops.append(stats[:, 0].cpu().numpy().copy())
    return feats.cpu().numpy(), np.stack(all_ids), np.stack(hops)


def exact_answers(idx, Qd, rec, k: int):
    import torch
    nq = Qd.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    cnt = torch.empty((nq,), dtype=torch.int32, device="cuda")
    jag.jag_exact_knn(idx, Qd, rec, k, ids, d2, cnt)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), cnt.cpu().numpy()


def targets_from(all_ids, exact_ids, exact_cnt, k: int, need: float = 0.95, unreachable: str = "widest"):
    """Per query, the smallest ladder index whose search reaches recall@k >=
    need.  A query that reaches it at no beam of the ladder gets the widest
    index (unreachable="widest"), or the smallest index at which its recall
    is highest over the ladder ("plateau": a wider beam finds it nothing
    more).  Which serves a workload better is measured: on the range
    workload the plateau rule saves work, on label-set workloads, whose
    recall keeps creeping up with the beam, the widest target does better.
    Returns (targets, reached)."""
    nl, nq, _ = all_ids.shape
    tgt = np.full(nq, nl - 1, dtype=np.int32)
    reached = np.zeros(nq, dtype=bool)
    for q in range(nq):
        den = min(k, int(exact_cnt[q]))
        if den == 0:
            tgt[q] = 0
            reached[q] = True
            continue
        gt = set(exact_ids[q, :den].tolist())
        hits = [len(gt.intersection(all_ids[i, q].tolist())) for i in range(nl)]
        ok = [i for i in range(nl) if hits[i] / den >= need]
        if ok:
            tgt[q] = ok[0]
            reached[q] = True
        elif unreachable == "plateau":
            tgt[q] = hits.index(max(hits))
    return tgt, reached


def fit(idx, Q, F, pool, k: int = 10, epochs: int = 40, batch: int = 512, lr: float = 3e-3,
        seed: int = 0, ladder=LADDER, exact_idx=None, rerank_mult: int = 0,
        dump: str | None = None, unreachable: str = "widest") -> tuple[np.ndarray, float, FitReport]:
    """Train on (Q, F) and attach the predictor to ``idx``.  ``exact_idx`` is an
    index over the same data holding an FP32 copy (defaults to ``idx``);
    ``rerank_mult`` must match the setting the learned search will use;
    ``unreachable`` is the target rule of queries that never reach recall 0.95
    (``targets_from``)."""
    import torch
    Qd, rec = _device_batch(idx, Q, F, pool)
    ex = exact_idx if exact_idx is not None else idx
    Qe, rece = (Qd, rec) if ex is idx else _device_batch(ex, Q, F, pool)
    exact_ids, exact_cnt = exact_answers(ex, Qe, rece, k)
    feats, all_ids, hops = traces(idx, Qd, rec, k, ladder, rerank_mult)
    tgt, reached = targets_from(all_ids, exact_ids, exact_cnt, k, unreachable=unreachable)
    if dump:
        nl, nq = all_ids.shape[0], all_ids.shape[1]
        hits = np.zeros((nl, nq), dtype=np.int8)
        for q in range(nq):
            gt = set(exact_ids[q, :min(k, int(exact_cnt[q]))].tolist())
            for i in range(nl):
                hits[i, q] = len(gt.intersection(all_ids[i, q].tolist()))
        np.savez_compressed(dump, features=feats, targets=tgt, reached=reached, hops=hops,
                            ladder=ladder, hits=hits, exact_cnt=exact_cnt)
    ok = feats[:, 15] == 1.0  # rows with four expansions
    X = torch.from_numpy(np.ascontiguousarray(feats[ok])).cuda()
    T = torch.from_numpy(tgt[ok].astype(np.float32)).cuda()
    P, loss = jag.jag_train_predictor(X, T, init_params(seed), epochs, batch, lr, seed)
    Ls = np.maximum(ladder[tgt], k).astype(np.float64)
    ratio = hops[tgt, np.arange(len(tgt))] / Ls
    rho = float(np.percentile(ratio[ok], 99)) if ok.any() else 8.0
    rho = max(rho, 1.0)
    jag.jag_set_predictor(idx, P, np.maximum(ladder, k), rho)
    rep = FitReport(int(ok.sum()), epochs, float(loss[0]), float(loss[-1]), rho,
                    np.bincount(tgt, minlength=len(ladder)).tolist(), int((~reached).sum()))
    return P, rho, rep
