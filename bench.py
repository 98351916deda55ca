"""Benchmark: filtered QPS at recall@10 = 0.95 per filter type on one MI355X.

One leg per (workload, filter type), all in the default run:
  range   -- 1,000,000 x 96, 256-cluster mixture, int32 attribute over
             [0, 10^6), 10,000 ranges of log-uniform selectivity, R = 64
             (the headline: timed steps, counters, the full CPU baseline);
  label   -- 20,000 x 32, 8 uniform labels, 10,000 label queries; and the
             serving shard, 1,250,000 x 100 with 1-5 Zipf labels of 1,000;
  subset  -- 1,000,000 x 128, 1-10 Zipf(1.1) labels of 1,000, subsets of
             1-3 labels (queries with at least k valid items);
  boolean -- the same items, (a AND b) OR c over Zipf labels.
Then the predictor at config-4 scale: 200,000 training traces of mixed
label/range/subset queries over the 20,000 x 32 vectors, scored on 10,000
held-out queries.

Per leg (untimed set-up): build the Threshold-JAG on the GPU, lay out FP32
and BF16 (+ FP32 copy) indexes over the same graph, compute the exact
answers with the CPU oracle (FP64), sweep the fixed beam L of each store,
fit the beam predictor on a separate query set of the same filter type,
sweep its offset for learned + BF16 + FP32-rerank search.  Each mode's
point is the smallest sweep beam or offset reaching recall >= 0.95 (grid
points, then bisection between the bracketing ones).  The operating point
(learned + BF16 where it reaches 0.95, else the fastest fixed mode) is
timed with HIP events (kernel path, records on the device) and end to end
through jag_search_batch (host filters); its roofline counts the bytes the
method must move.  The headline's timed steps run its operating point over
the whole query batch, inputs resident in HBM.  One JSON line on stdout.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--legs c2:range,...]
                    [--config c1|c2|c3|c5|bool15] [--no-c4]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "filtered QPS at recall@10=0.95 per filter type, learned+BF16 vs plain FP32 on 1 GPU"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=None,
                    help="run only this workload's legs (default: every leg of --legs)")
    ap.add_argument("--legs", default="c2:range,c1:label,c3:subset,c3:boolean,c5:label,c5:serve",
                    help="workload:filter-type legs; the first is the headline (timed steps, "
                         "counters, full CPU baseline); c5:serve is the serving leg (Poisson "
                         "arrivals, batch and slot admission)")
    ap.add_argument("--serve-rates", default="25000,100000,200000",
                    help="offered rates of the serving leg (requests/s)")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="arrivals per rate and admission mode of the serving leg (seconds)")
    ap.add_argument("--serve-queries", type=int, default=4000,
                    help="distinct mixed queries of the serving leg (exact answers from the oracle)")
    ap.add_argument("--no-c4", action="store_true", help="skip the predictor evaluation at 200k traces")
    ap.add_argument("--c4-train", type=int, default=200000)
    ap.add_argument("--c4-heldout", type=int, default=10000)
    ap.add_argument("--leg-cpu-seconds", type=float, default=3.0,
                    help="CPU baseline time per non-headline leg")
    ap.add_argument("--n", type=int, default=None, help="override the number of vectors")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--ntrain", type=int, default=20000)
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU baseline over its sample for about this long")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-fixed", action="store_true")
    ap.add_argument("--profile-op", action="store_true",
                    help="run only the operating point (for rocprofv3); needs --L and --store")
    ap.add_argument("--L", type=int, default=48)
    ap.add_argument("--op-mode", default="fp32-fixed",
                    choices=["fp32-fixed", "bf16+rerank-fixed", "fp8+rerank-fixed", "learned+bf16+rerank"])
    ap.add_argument("--delta", type=float, default=0.0)
    ap.add_argument("--single-pass", action="store_true",
                    help="profile mode, learned: the one-pass schedule (prediction inside the search)")
    ap.add_argument("--ladder", default=None,
                    help="profile mode, learned: comma-separated ladder (as the bench line reports it)")
    ap.add_argument("--target-rule", default="widest", choices=["widest", "plateau"],
                    help="profile mode, learned: training target of queries that never reach recall 0.95 "
                         "(as the bench line reports it)")
    ap.add_argument("--ladder-top", type=int, default=None,
                    help="widest beam of the learned ladder (default: 1.4x the fixed beam at recall 0.95)")
    ap.add_argument("--dump-traces", default=None, help="save predictor traces to this .npz")
    ap.add_argument("--serve", action="store_true", help="serving benchmark (Poisson arrivals)")
    ap.add_argument("--rates", default="5000,20000,50000,100000,200000")
    ap.add_argument("--admission", default="both", choices=["slots", "batches", "both"],
                    help="--serve: how the server admits requests (resident waves, batches per stream, or both "
                         "one after the other)")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="profile mode: also run device copies of this many bytes")
    ap.add_argument("--min-valid", type=int, default=None,
                    help="drop queries with fewer valid items (default: k for the label-set "
                         "workloads c3 and c5, else 0)")
    ap.add_argument("--filter-type", type=int, default=None, choices=[0, 1, 2, 3, 4],
                    help="profile mode: keep only the queries of this filter type "
                         "(0 label, 1 range, 2 subset, 3 Boolean)")
    ap.add_argument("--build", default="device", choices=["device", "host", "both"],
                    help="where the graph is built (both: host and device, checked equal, both timed)")
    ap.add_argument("--R", type=int, default=0, help="out-degree bound of the graph (default: the workload's)")
    ap.add_argument("--thresholds", default=None,
                    help="comparator list of the build, e.g. 'labels:1,labels:0.01,labels:0' or "
                         "'weight:labels:0,weight:labels:1,weight:labels:10' (default: the workload's)")
    ap.add_argument("--build-only", action="store_true",
                    help="build the workload's graph (see --build), print the build times, exit")
    ap.add_argument("--graph-cache", default=None,
                    help="load the graph from this .npz if present, else build and save it there")
    return ap.parse_args()


def build_graph(args, w, thresholds):
    """The workload's graph on the GPU and/or host threads (the same graph);
    returns (adj, entry, {where: seconds})."""
    from paper_2602_10258_amd import jag
    kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab, R=w.R, L_build=2 * w.R,
              thresholds=thresholds, seed=0, progress=True)
    times, out = {}, {}
    for where in (["host", "device"] if args.build == "both" else [args.build]):
        t = time.time()
        out[where] = jag.jag_build_graph(w.X, device=where == "device", **kw)
        times[where] = round(time.time() - t, 2)
        log(f"graph built on the {where} in {times[where]:.2f}s")
    if len(out) == 2:
        same = out["host"][1] == out["device"][1] and np.array_equal(out["host"][0], out["device"][0])
        log(f"host and device graphs identical: {same}")
        assert same, "the device builder must give the host builder's graph"
    adj, entry = out["device" if "device" in out else "host"]
    return adj, entry, times


class Timer:
    """HIP events on torch's current stream, which is the stream the searches use."""

    def __init__(self):
        import torch
        self.torch = torch

    def run(self, fn, reps: int, warm: int = 1):
        t = self.torch
        for _ in range(warm):
            fn()
        t.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.median(times))


FILTER_NAMES = {0: "label", 1: "range", 2: "subset", 3: "boolean", 4: "boolean-table"}

# beams of the fixed-beam sweeps (the kernel takes up to 1024)
LADDER_FIXED = [10, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 56, 64, 80, 96, 128, 192, 256, 384, 512,
                768, 1024]


def learned_ladder(L95, top=None):
    """Beams the predictor chooses from, sized to the workload: up to the
    smallest sweep beam >= 1.4x the fixed beam that reaches recall 0.95 (at
    least 64, all of them if none does; `top` overrides), at most 16 entries
    spaced evenly in log scale.  On the range workload this gives a ladder
    topping at 64, which measured better than one to 128."""
    if top is None:
        top = 1024 if L95 is None else next((L for L in LADDER_FIXED if L >= max(64, 1.4 * L95)), 1024)
    cand = [L for L in LADDER_FIXED if L <= top]
    if len(cand) > 16:
        want = np.exp(np.linspace(np.log(cand[0]), np.log(top), 16))
        cand = sorted({min(cand, key=lambda L: abs(np.log(L) - np.log(x))) for x in want})
    return np.array(cand, dtype=np.int32)

def ladder_tops(L95, top=None):
    """Widest ladder beams to try, narrowest first; the bench keeps the first
    whose learned sweep reaches recall 0.95.  A narrow top keeps the widest
    searches' lists short (more of them fit on the device at once), but a
    top at the fixed beam itself can leave the learned search just below
    0.95.  From max(64, that fixed beam) up to the default top."""
    if top is not None:
        return [top]
    if L95 is None:
        return [None]
    hi = int(learned_ladder(L95)[-1])
    return [L for L in LADDER_FIXED if max(64, L95) <= L <= hi] or [hi]


# (attribute kind, quantile) lists: 0 scalar, 1 labels |a XOR b|, 2 labels with
# the frequency-weighted distance the paper uses for skewed label vocabularies
THRESHOLDS = {
    "c1": [(1, 1.0), (1, 0.0)],
    "c2": [(0, 1.0), (0, 0.01), (0, 0.0)],
    "c3": [(2, 1.0), (2, 0.01), (2, 0.0)],
    "c5": [(0, 1.0), (0, 0.01), (0, 0.0), (2, 0.01), (2, 0.0)],
    # 15 binary variables as labels: |a XOR b| is the Hamming distance of assignments
    "bool15": [(1, 1.0), (1, 0.01), (1, 0.0)],
}


KIND_NAMES = {"scalar": 0, "labels": 1, "wlabels": 2}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse_thresholds(text: str):
    """'labels:1,labels:0.01,labels:0' -> [(1, 1.0), (1, 0.01), (1, 0.0)];
    a 'weight:' prefix makes a Weight-JAG entry (value = the multiplier)."""
    out = []
    for item in text.split(","):
        parts = item.strip().split(":")
        weight = parts[0] == "weight"
        if weight:
            parts = parts[1:]
        if len(parts) != 2 or parts[0] not in KIND_NAMES:
            raise SystemExit(f"bad threshold entry {item!r}: want [weight:]scalar|labels|wlabels:value")
        out.append((KIND_NAMES[parts[0]] | (0x100 if weight else 0), float(parts[1])))
    return out


KERNEL_SOURCES = ("search_device.h", "search.hip")


def kernel_source_sha1() -> str:
    """sha1 over the search kernel's sources (the device code, then its launches)."""
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2602_10258_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str, op_name: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summaries (one entry, or a list of entries, one per operating point),
    only if taken on this exact kernel source and operating point;
    otherwise None."""
    p = os.path.join(ROOT, "profiles", f"search_kernel_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    sha = kernel_source_sha1()
    for e in d if isinstance(d, list) else [d]:
        if e.get("kernel_source_sha1") == sha and e.get("operating_point") == op_name:
            return e["traffic_bytes_per_launch"]
    return None


def serve_main(args):
    """Serving: Poisson arrivals of mixed Label/Range/Subset/Boolean queries on
    one GPU's shard of the 10M-vector serving workload (FP8 store + FP32
    rerank, learned beam).  Prints one JSON line with p50/p99 latency and the
    achieved QPS per offered rate."""
    import torch
    from oracle import oracle as O
    from paper_2602_10258_amd import jag
    from paper_2602_10258_amd import predictor as pred
    from workloads import make_config
    from workloads.gen import extra_queries, poisson_arrivals

    n = args.n or 1_250_000
    w = make_config("c5", n=n, nq=args.nq or 10000)
    if args.R:
        w = dataclasses.replace(w, R=args.R)
    k = w.k
    log(f"serving workload c5 shard: n={w.n} d={w.d} nq={w.nq}")
    t1 = time.time()
    if args.graph_cache and os.path.exists(args.graph_cache):
        z = np.load(args.graph_cache)
        adj, entry = z["adj"], int(z["entry"])
    else:
        adj, entry, _ = build_graph(args, w, THRESHOLDS["c5"])
        if args.graph_cache:
            np.savez(args.graph_cache, adj=adj, entry=entry)
    log(f"graph ready in {time.time() - t1:.1f}s")
    kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    ix = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_FP8_E4M3, keep_f32=True, **kw)
    Qt, Ft, pt = extra_queries(w, args.ntrain, qseed=1000)
    nthr = min(os.cpu_count() or 1, 16)
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, k, nthreads=nthr)
    keep = nv >= (args.min_valid if args.min_valid is not None else k)
    log(f"keeping {int(keep.sum())} of {len(keep)} queries with >= k valid items")
    w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
    gi, gd, nv = gi[keep], gd[keep], nv[keep]

    def recall_of(ids_np):
        r = []
        for q in range(len(ids_np)):
            den = min(k, int(nv[q]))
            if den:
                r.append(len(set(gi[q, :den].tolist()) & set(ids_np[q].tolist())) / den)
        return float(np.mean(r))

    # the fixed beam that reaches recall 0.95 sizes the predictor's ladder
    dev = torch.device("cuda:0")
    rec = torch.from_numpy(jag.jag_encode_filters(ix, w.F, w.pool)).to(dev)
    Qd = torch.from_numpy(w.Q).to(dev)
    ids = torch.empty((w.nq, k), dtype=torch.int32, device=dev)
    dd = torch.empty((w.nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((w.nq,), dtype=torch.int32, device=dev)
    L95 = None
    for L in LADDER_FIXED:
        jag.jag_search_encoded(ix, Qd, rec, k, jag.SearchParams(L=L, rerank_mult=4), ids, dd, cnt)
        torch.cuda.synchronize()
        if recall_of(ids.cpu().numpy()) >= 0.95:
            L95 = L
            break
    # the narrowest ladder top whose learned search reaches 0.95 on the
    # batch path (as in the main sweep); the smallest offset reaching it
    delta = None
    for top in ladder_tops(L95, args.ladder_top):
        lad = learned_ladder(L95, top)
        log(f"fixed beam at recall 0.95: {L95}; learned ladder {lad.tolist()}")
        _, rho, rep = pred.fit(ix, Qt, Ft, pt, k=k, rerank_mult=4, ladder=lad)
        log(f"predictor: loss {rep.loss_first:.2f} -> {rep.loss_last:.2f}, rho {rho:.2f}")
        for dl in [-1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]:
            sp = jag.SearchParams(L=k, learned=1, delta=dl, rerank_mult=4)
            jag.jag_search_encoded(ix, Qd, rec, k, sp, ids, dd, cnt)
            torch.cuda.synchronize()
            r = recall_of(ids.cpu().numpy())
            log(f"delta {dl:+.1f}: batch recall {r:.4f}")
            if r >= 0.95:
                delta = dl
                break
        if delta is not None:
            break
    if delta is None:
        delta = 6.0
    sp = jag.SearchParams(L=k, learned=1, delta=delta, rerank_mult=4)
    rates = [float(x) for x in args.rates.split(",")]
    per_rate = []
    modes = ["batches", "slots"] if args.admission == "both" else [args.admission]
    for mode in modes:
        for qps in rates:
            m = max(2000, int(qps * args.serve_seconds))
            arr = poisson_arrivals(np.random.default_rng(int(qps)), m, qps)
            if mode == "slots":
                s = jag.jag_server_start(ix, k, sp, slot_admission=True)
            else:
                s = jag.jag_server_start(ix, k, sp, max_batch=4096, n_streams=4, max_wait_us=100)
            try:
                got, st = poisson_run(jag, s, w.Q, w.F, w.pool, arr, k)
            finally:
                jag.jag_server_stop(s)
            qi = np.arange(m) % w.nq
            r = float(np.mean([len(set(gi[q, :min(k, int(nv[q]))].tolist()) & set(got[i].tolist()))
                               / max(1, min(k, int(nv[q]))) for i, q in enumerate(qi)]))
            row = {"admission": mode, "offered_qps": qps, "requests": m, "achieved_qps": round(st["qps"], 1),
                   "p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
                   "max_ms": round(st["max_us"] / 1e3, 3), "launches": st["batches"],
                   "max_inflight": st["max_inflight_seen"], "resident_capacity": st["resident_capacity"],
                   "recall_at_10": round(r, 4)}
            log(row)
            per_rate.append(row)
    out = {"metric": "serving latency (p50/p99) and QPS, mixed filters, learned beam + FP8 + FP32 rerank",
           "config": {"workload": f"c5: {w.n} x {w.d}, FP8 E4M3 + per-row scale, "
                                  f"R={w.R}, mixed Label/Range/Subset/Boolean, Poisson arrivals",
                      "queries": w.nq, "delta": delta, "rho": rho, "ladder": lad.tolist() if lad is not None else None},
           "rates": per_rate}
    print(json.dumps(out), flush=True)


def poisson_run(jag, s, Q, F, pool, arrivals, k):
    """Submit request i at arrivals[i] (seconds from now; query i mod len(Q)),
    wait for all, return (ids[m, k], server stats)."""
    m, nq = len(arrivals), len(Q)
    qi = np.arange(m) % nq
    t0 = time.perf_counter()
    tick = np.empty(m, dtype=np.uint64)
    i = 0
    while i < m:
        now = time.perf_counter() - t0
        j = int(np.searchsorted(arrivals, now, side="right"))
        if j > i:
            tick[i:j] = jag.jag_server_submit(s, Q[qi[i:j]], F[qi[i:j]], pool)
            i = j
        else:
            time.sleep(max(0.0, min(1e-4, arrivals[i] - now)))
    jag.jag_server_drain(s)
    st = jag.jag_server_stats_get(s)
    got = np.empty((m, k), dtype=np.int32)
    for q in range(m):
        got[q] = jag.jag_server_poll(s, int(tick[q]))[0]
    return got, st


def serve_leg(args, cfg):
    """Serving on the shard workload: Poisson arrivals of mixed Label, Range,
    Subset and Boolean queries at a few offered rates, the learned beam (one
    pass) over the FP8 store with the FP32 rerank at recall 0.95, through the
    server with batch admission and with slot admission (resident waves that
    take one request at a time).  p50/p99 latency from submit to the host
    seeing the answer, per rate and admission mode."""
    from oracle import oracle as O
    from paper_2602_10258_amd import jag
    from paper_2602_10258_amd import predictor as pred
    from workloads.gen import extra_queries, poisson_arrivals
    torch = cfg.torch
    w, k, dev = cfg.w, cfg.w.k, cfg.dev
    t0 = time.time()
    ix = cfg.ix8()
    Q, F, pool = extra_queries(w, args.serve_queries, qseed=7000)
    gi, _, nv = O.bruteforce(w.X, cfg.A, Q, F, pool, k, nthreads=cfg.nthr)
    keep = nv >= k
    Q, F, gi, nv = np.ascontiguousarray(Q[keep]), np.ascontiguousarray(F[keep]), gi[keep], nv[keep]
    nq = len(Q)
    log(f"[serve] {nq} mixed queries with >= k valid items, exact answers in {time.time() - t0:.1f}s")

    def recall_of(ids_np, qi):
        return float(np.mean([len(set(gi[q, :k].tolist()) & set(ids_np[i].tolist())) / k
                              for i, q in enumerate(qi)]))

    rec = torch.from_numpy(jag.jag_encode_filters(ix, F, pool)).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dd = torch.empty((nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((nq,), dtype=torch.int32, device=dev)
    allq = np.arange(nq)

    def batch_recall(sp):
        jag.jag_search_encoded(ix, Qd, rec, k, sp, ids, dd, cnt)
        torch.cuda.synchronize()
        return recall_of(ids.cpu().numpy(), allq)

    L95 = next((L for L in LADDER_FIXED if batch_recall(jag.SearchParams(L=L, rerank_mult=4)) >= 0.95), None)
    Qt, Ft, pt = extra_queries(w, args.ntrain, qseed=1000)
    delta, lad, rho = None, None, None
    for top in ladder_tops(L95, args.ladder_top):
        lad = learned_ladder(L95, top)
        _, rho, rep = pred.fit(ix, Qt, Ft, pt, k=k, rerank_mult=4, ladder=lad)
        for dl in [0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0]:
            r = batch_recall(jag.SearchParams(L=k, learned=1, delta=dl, rerank_mult=4, single_pass=1))
            if r >= 0.95:
                delta = dl
                break
        if delta is not None:
            break
    delta = 6.0 if delta is None else delta
    sp = jag.SearchParams(L=k, learned=1, delta=delta, rerank_mult=4)
    log(f"[serve] fixed beam at 0.95: {L95}; ladder {lad.tolist()}, delta {delta}, rho {rho:.2f}")
    rows = []
    for mode in ("batches", "slots"):
        for qps in [float(x) for x in args.serve_rates.split(",")]:
            m = max(3000, int(qps * args.serve_seconds))
            arr = poisson_arrivals(np.random.default_rng(int(qps)), m, qps)
            if mode == "slots":
                s = jag.jag_server_start(ix, k, sp, slot_admission=True)
            else:
                s = jag.jag_server_start(ix, k, sp, max_batch=4096, n_streams=4, max_wait_us=100)
            try:
                got, st = poisson_run(jag, s, Q, F, pool, arr, k)
            finally:
                jag.jag_server_stop(s)
            row = {"admission": mode, "offered_qps": qps, "requests": m, "achieved_qps": round(st["qps"], 1),
                   "p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
                   "max_ms": round(st["max_us"] / 1e3, 3), "launches": st["batches"],
                   "max_inflight": st["max_inflight_seen"], "resident_capacity": st["resident_capacity"],
                   "recall_at_10": round(recall_of(got, np.arange(m) % nq), 4)}
            log(f"[serve] {row}")
            rows.append(row)
    return {"workload": f"{w.name} shard: {w.n} x {w.d}, FP8 E4M3 + row scale + FP32 rerank, R={w.R}, "
                        f"equal mix of label/range/subset/Boolean filters, Poisson arrivals",
            "queries": nq, "fixed_L_at_095": L95, "ladder": lad.tolist(), "delta": delta, "rho": round(rho, 3),
            "rates": rows, "seconds": round(time.time() - t0, 1)}


FILTER_CODES = {"label": 0, "range": 1, "subset": 2, "boolean": 3, "table": 4}
STORE_NAMES = {0: "fp32", 1: "bf16 (+fp32 rerank)", 2: "fp8 e4m3 + row scale (+fp32 rerank)"}


def attr_bytes(w, ftype: int) -> int:
    """Attribute bytes one fresh neighbour costs the method: the int32 scalar
    of a range filter, else the item's labels as uint16 (up to the
    workload's largest label count)."""
    if ftype == 1:
        return 4
    return 2 * int(np.max(np.diff(w.loff)))


def row_bytes(d: int, store: int) -> int:
    return d * {0: 4, 1: 2, 2: 1}[store] + (4 if store == 2 else 0)


def rounded(r: dict) -> dict:
    return {k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in r.items()}


class Config:
    """One workload: its graph, FP32 and BF16 (+ FP32 copy) indexes over the
    same graph, and the oracle's exact answers of its queries."""

    def __init__(self, args, name, dev, types=None):
        import torch
        from oracle import oracle as O
        from paper_2602_10258_amd import jag
        from workloads import make_config
        self.name = name
        t0 = time.time()
        n = args.n if args.n else (1_250_000 if name == "c5" else None)
        # the serving shard's queries mix four filter types: draw enough that
        # each type a leg needs keeps about 10,000
        if args.nq:
            nq = args.nq
        elif name == "c5":
            nq = 40000 // len(types) if types else 10000
        else:
            nq = 10000 if name == "c1" else None
        w = make_config(name, n=n, nq=nq)
        if args.R:
            w = dataclasses.replace(w, R=args.R)
        if types is not None:
            keep = np.isin(w.F[:, 0], types)
            w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
        self.thr = parse_thresholds(args.thresholds) if args.thresholds else THRESHOLDS[w.name]
        log(f"workload {w.name}: n={w.n} d={w.d} nq={w.nq} ({time.time() - t0:.1f}s)")
        t1 = time.time()
        cache = args.graph_cache and args.graph_cache.replace("{config}", name)
        if cache and os.path.exists(cache):
            z = np.load(cache)
            self.adj, self.entry, self.build_times = z["adj"], int(z["entry"]), {"cached": 0.0}
        else:
            self.adj, self.entry, self.build_times = build_graph(args, w, self.thr)
            if cache:
                np.savez(cache, adj=self.adj, entry=self.entry)
        self.build_s = time.time() - t1
        log(f"graph of {name} ready in {self.build_s:.1f}s, mean degree {(self.adj >= 0).sum(1).mean():.1f}")
        self.kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab)
        self.ix32 = jag.jag_build_from_graph(w.X, self.adj, self.entry, store=jag.STORE_F32, **self.kw)
        self.ix16 = jag.jag_build_from_graph(w.X, self.adj, self.entry, store=jag.STORE_BF16, keep_f32=True,
                                             **self.kw)
        self._ix8 = None
        # ground truth: the oracle's exact filtered k-NN in FP64
        t2 = time.time()
        self.nthr = min(os.cpu_count() or 1, 16)
        self.A = O.attrs_of(w)
        gi, gd, nv = O.bruteforce(w.X, self.A, w.Q, w.F, w.pool, w.k, nthreads=self.nthr)
        log(f"exact answers of {name} (oracle, {self.nthr} threads) in {time.time() - t2:.1f}s")
        min_valid = args.min_valid if args.min_valid is not None else (w.k if name in ("c3", "c5") else 0)
        keep = nv >= min_valid
        if not keep.all():
            # label-set workloads keep only queries with at least k valid items
            log(f"keeping {int(keep.sum())} of {len(keep)} queries with >= {min_valid} valid items")
            w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
            gi, gd, nv = gi[keep], gd[keep], nv[keep]
        self.w, self.gi, self.nv = w, gi, nv
        self.dev = dev
        self.torch = torch

    def ix8(self):
        from paper_2602_10258_amd import jag
        if self._ix8 is None:
            w = self.w
            self._ix8 = jag.jag_build_from_graph(w.X, self.adj, self.entry, store=jag.STORE_FP8_E4M3,
                                                 keep_f32=True, **self.kw)
        return self._ix8

    def describe(self) -> str:
        w = self.w
        return (f"{w.name}: {w.n} x {w.d} clustered vectors ({w.meta.get('thresholds')}), k={w.k}, R={w.R}")


class Leg:
    """The queries of one filter type of a workload, on the device, with their
    exact answers; sweeps and timings of every search mode over them."""

    def __init__(self, cfg: Config, ftype: int, timer):
        from paper_2602_10258_amd import jag
        torch = cfg.torch
        sel = np.flatnonzero(cfg.w.F[:, 0] == ftype)
        assert len(sel), f"no {FILTER_NAMES[ftype]} queries in {cfg.name}"
        self.cfg, self.ftype, self.timer = cfg, ftype, timer
        self.Q = np.ascontiguousarray(cfg.w.Q[sel])
        self.F = np.ascontiguousarray(cfg.w.F[sel])
        self.pool = cfg.w.pool
        self.gi, self.nv = cfg.gi[sel], cfg.nv[sel]
        self.nq, self.k = len(sel), cfg.w.k
        dev = cfg.dev
        self.Qd = torch.from_numpy(self.Q).to(dev)
        self.rec = {id(cfg.ix32): torch.from_numpy(jag.jag_encode_filters(cfg.ix32, self.F, self.pool)).to(dev),
                    id(cfg.ix16): torch.from_numpy(jag.jag_encode_filters(cfg.ix16, self.F, self.pool)).to(dev)}
        self.ids = torch.empty((self.nq, self.k), dtype=torch.int32, device=dev)
        self.d2 = torch.empty((self.nq, self.k), dtype=torch.float32, device=dev)
        self.cnt = torch.empty((self.nq,), dtype=torch.int32, device=dev)
        self.stats = torch.zeros((self.nq, 4), dtype=torch.int32, device=dev)
        self.has_valid = self.nv > 0

    def distance_error(self) -> dict:
        """Relative error of the returned squared distances (the last search's
        outputs) against the FP64 distances of the same ids."""
        X = self.cfg.w.X
        ids, d2, cnt = self.ids.cpu().numpy(), self.d2.cpu().numpy(), self.cnt.cpu().numpy()
        valid = np.arange(ids.shape[1])[None, :] < cnt[:, None]
        safe = np.where(valid, ids, 0)
        exact = ((X[safe].astype(np.float64) - self.Q[:, None, :].astype(np.float64)) ** 2).sum(-1)
        rel = np.abs(d2.astype(np.float64) - exact) / np.maximum(exact, 1e-30)
        rel = rel[valid]
        if rel.size == 0:
            return None
        return {"results": int(rel.size), "mean_rel": float(f"{rel.mean():.3e}"), "max_rel": float(f"{rel.max():.3e}")}

    def selectivity_accuracy(self) -> dict:
        """The records' selectivity estimate (a predictor feature) against the
        exact fraction of valid items (from the oracle's exact answers), over
        queries with at least one valid item: mean and 90th percentile of
        |log2(estimate / exact)|, and the correlation of the two logs."""
        # the records (truth-table filters append their distance tables after them)
        rec = self.rec[id(self.cfg.ix32)].cpu().numpy().reshape(-1)[:self.nq * 128].reshape(self.nq, 128)
        est = rec[:, 28:32].copy().view(np.float32)[:, 0].astype(np.float64)
        ok = self.nv > 0
        if not ok.any():
            return None
        exact = self.nv[ok] / float(self.cfg.w.n)
        le, lx = np.log2(np.maximum(est[ok], 1e-12)), np.log2(exact)
        err = np.abs(le - lx)
        corr = float(np.corrcoef(le, lx)[0, 1]) if np.std(le) > 0 and np.std(lx) > 0 else None
        return {"queries": int(ok.sum()), "mean_abs_log2_error": round(float(err.mean()), 4),
                "p90_abs_log2_error": round(float(np.percentile(err, 90)), 4),
                "log_correlation": corr and round(corr, 4)}

    def records(self, ix):
        from paper_2602_10258_amd import jag
        if id(ix) not in self.rec:
            self.rec[id(ix)] = self.cfg.torch.from_numpy(jag.jag_encode_filters(ix, self.F, self.pool)).to(self.cfg.dev)
        return self.rec[id(ix)]

    def recall(self, ids_np) -> float:
        hits = np.zeros(self.nq)
        for q in range(self.nq):
            den = min(self.k, int(self.nv[q]))
            if den:
                hits[q] = len(set(self.gi[q, :den].tolist()) & set(ids_np[q].tolist())) / den
        return float(hits[self.has_valid].mean())

    def search(self, ix, sp):
        from paper_2602_10258_amd import jag
        jag.jag_search_encoded(ix, self.Qd, self.records(ix), self.k, sp, self.ids, self.d2, self.cnt)

    def point(self, ix, sp) -> dict:
        from paper_2602_10258_amd import jag
        ms = self.timer.run(lambda: self.search(ix, sp), reps=7, warm=1)
        self.search(ix, jag.SearchParams(**{**sp.__dict__, "stats": self.stats}))
        self.cfg.torch.cuda.synchronize()
        st = self.stats.cpu().numpy()
        return dict(ms=ms, qps=self.nq / (ms / 1e3), recall=self.recall(self.ids.cpu().numpy()),
                    hops=float(st[:, 0].mean()), ndist=float(st[:, 1].mean()), nattr=float(st[:, 2].mean()),
                    lhat=float(st[:, 3].mean()))

    def fixed_sweep(self, ix, label, rerank_mult=0, beams=None):
        from paper_2602_10258_amd import jag
        curve = []
        for L in beams or LADDER_FIXED:
            r = self.point(ix, jag.SearchParams(L=L, rerank_mult=rerank_mult))
            r["L"] = L
            curve.append(r)
            log(f"{self.tag()} {label} L={L:4d} recall={r['recall']:.4f} qps={r['qps']:.0f} hops={r['hops']:.1f}")
            if r["recall"] >= 0.99:
                break
        # bisect the integer beams between the last grid point below recall
        # 0.95 and the first at or above it: the measured point is the
        # smallest beam reaching 0.95, not the next grid beam
        j = next((i for i, r in enumerate(curve) if r["recall"] >= 0.95), None)
        if j:
            lo, hi = curve[j - 1]["L"], curve[j]["L"]
            while hi - lo > 1:
                mid = (lo + hi) // 2
                r = self.point(ix, jag.SearchParams(L=mid, rerank_mult=rerank_mult))
                r["L"] = mid
                curve.append(r)
                log(f"{self.tag()}   refine L={mid:4d} recall={r['recall']:.4f} qps={r['qps']:.0f}")
                lo, hi = (lo, mid) if r["recall"] >= 0.95 else (mid, hi)
            curve.sort(key=lambda r: r["L"])
        return curve

    def learned_sweep(self, ntrain, L95, ladder_top=None, dump=None, ix=None, tag="bf16"):
        """Fit the predictor on a separate query set of this filter type and
        sweep its offset; the narrowest ladder whose sweep reaches 0.95.  Both
        target rules for training queries that never reach 0.95 (the widest
        beam, or the beam where their recall peaks) are fitted and swept; the
        one with the higher QPS at 0.95 stays attached to the index (``ix``,
        the BF16 index by default)."""
        from paper_2602_10258_amd import jag
        from paper_2602_10258_amd import predictor as pred
        from workloads.gen import extra_queries
        cfg = self.cfg
        ix = cfg.ix16 if ix is None else ix
        t3 = time.time()
        Qt, Ft, pt = extra_queries(cfg.w, ntrain * (2 if cfg.name == "c3" else 4 if cfg.name == "c5" else 1),
                                   qseed=1000)
        keep = Ft[:, 0] == self.ftype
        Qt, Ft = np.ascontiguousarray(Qt[keep][:ntrain]), np.ascontiguousarray(Ft[keep][:ntrain])

        def sweep(rule):
            learned, lad, rep, P, rho = [], None, None, None, None
            for top in ladder_tops(L95, ladder_top):
                lad = learned_ladder(L95, top)
                log(f"{self.tag()} learned ladder {lad.tolist()}, unreachable targets: {rule}")
                P, rho, rep = pred.fit(ix, Qt, Ft, pt, k=self.k, exact_idx=cfg.ix32, rerank_mult=4,
                                       dump=dump, ladder=lad, unreachable=rule)
                log(f"{self.tag()} predictor fitted on {rep.n_train} traces in {time.time() - t3:.1f}s: loss "
                    f"{rep.loss_first:.3f} -> {rep.loss_last:.3f}, rho={rho:.2f}, unreachable={rep.unreachable}")
                learned = []
                for delta in [-1.0, -0.5, 0.0, 0.5, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 4.0, 6.0]:
                    r = self.point(ix, jag.SearchParams(L=self.k, learned=1, delta=delta, rerank_mult=4))
                    r["delta"] = delta
                    learned.append(r)
                    log(f"{self.tag()} learned+{tag} delta={delta:+.2f} recall={r['recall']:.4f} "
                        f"qps={r['qps']:.0f} mean Lhat={r['lhat']:.1f}")
                    if r["recall"] >= 0.995 or (r["recall"] >= 0.95 and delta >= 1.0):
                        break
                if any(r["recall"] >= 0.95 for r in learned):
                    break
            # bisect the offset between the last point below 0.95 and the first
            # at or above it (four halvings; midpoints rounded to 4 decimals)
            j = next((i for i, r in enumerate(learned) if r["recall"] >= 0.95), None)
            if j:
                lo, hi = learned[j - 1]["delta"], learned[j]["delta"]
                for _ in range(4):
                    mid = round((lo + hi) / 2, 4)
                    r = self.point(ix, jag.SearchParams(L=self.k, learned=1, delta=mid, rerank_mult=4))
                    r["delta"] = mid
                    learned.append(r)
                    log(f"{self.tag()}   refine delta={mid:+.4f} recall={r['recall']:.4f} qps={r['qps']:.0f}")
                    lo, hi = (lo, mid) if r["recall"] >= 0.95 else (mid, hi)
                learned.sort(key=lambda r: r["delta"])
            return learned, lad, rep, P, rho

        runs = {rule: sweep(rule) for rule in ("widest", "plateau")}

        def score(run):
            best = at95(run[0])[0]
            return best["qps"] if best else -1.0
        rule = max(runs, key=lambda r: score(runs[r]))
        learned, lad, rep, P, rho = runs[rule]
        if P is not None:
            jag.jag_set_predictor(ix, P, np.maximum(lad, self.k), rho)
        rules = {r: round(score(v), 1) if score(v) > 0 else None for r, v in runs.items()}
        if tag == "bf16":
            self.target_rules, self.target_rule = rules, rule
        log(f"{self.tag()} learned+{tag} QPS at 0.95 by target rule: {rules}; keeping {rule}")
        return learned, lad, rep

    def tag(self):
        return f"[{self.cfg.name}:{FILTER_NAMES[self.ftype]}]"

    def alg_bytes(self, st, store, rerank) -> float:
        """Sum over the batch of the bytes the method must move per query:
        per expansion the R neighbour ids, an attribute per fresh neighbour and
        a row per distance, plus the query, its record, the outputs and the
        rerank rows."""
        w = self.cfg.w
        per_q = (st[:, 0] * 4 * w.R + st[:, 2] * attr_bytes(w, self.ftype) + st[:, 1] * row_bytes(w.d, store)
                 + 4 * w.d + 128 + 8 * self.k + 4)
        if rerank:
            per_q = per_q + 4 * self.k * 4 * w.d
        return float(per_q.sum())

    def op_measure(self, ix, sp, store, rerank, reps=7):
        """Kernel time (median of HIP-event launches), roofline, and the end-to-end
        rate from host filters (jag_search_batch: encoding, pinned staging and the
        record upload included; query vectors and outputs on the device)."""
        from paper_2602_10258_amd import jag
        torch = self.cfg.torch
        kern_ms = self.timer.run(lambda: self.search(ix, sp), reps=reps, warm=2)
        self.search(ix, jag.SearchParams(**{**sp.__dict__, "stats": self.stats}))
        torch.cuda.synchronize()
        st = self.stats.cpu().numpy().astype(np.int64)
        alg = self.alg_bytes(st, store, rerank)
        achieved = alg / (kern_ms / 1e3) / 1e9

        def host():
            jag.jag_search_batch(ix, self.Qd, self.F, self.pool, self.k, sp, self.ids, self.d2, self.cnt)
        host()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            host()
        torch.cuda.synchronize()
        e2e = self.nq * reps / (time.perf_counter() - t)
        return dict(kernel_ms=round(kern_ms, 4), kernel_qps=round(self.nq / (kern_ms / 1e3), 1),
                    end_to_end_qps=round(e2e, 1), distance_error=self.distance_error(),
                    roofline={"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": round(achieved / PEAK_HBM_GBS, 4),
                              "gather_ceiling": gather_ceiling(self.cfg, self, st, store, rerank, achieved)},
                    alg_bytes_per_query=round(alg / self.nq, 1), mean_expansions=round(float(st[:, 0].mean()), 2),
                    mean_distance_computations=round(float(st[:, 1].mean()), 2),
                    mean_attribute_evaluations=round(float(st[:, 2].mean()), 2))

    def cpu(self, L, seconds, sample):
        """The oracle (FP64, plain FP32 fixed beam L) on the machine's host cores over
        whole passes of a bounded sample of these queries."""
        from oracle import oracle as O
        cfg = self.cfg
        m = min(sample, self.nq)
        reps, cs = 0, 0.0
        while reps == 0 or cs < seconds:
            t4 = time.time()
            O.search(cfg.w.X, cfg.adj, cfg.entry, cfg.A, self.Q[:m], self.F[:m], self.pool, L, self.k,
                     nthreads=cfg.nthr)
            cs += time.time() - t4
            reps += 1
        return {"value": round(reps * m / cs, 1), "unit": "queries/s", "cores": cfg.nthr, "kind": "oracle",
                "sample": f"{m} of the {self.nq} {FILTER_NAMES[self.ftype]} queries of {cfg.name}, {reps} passes, "
                          f"plain FP32 fixed beam L={L}, FP64 distances, {cs:.1f}s"}


def at95(curve):
    """The first sweep point (smallest beam or offset) at or above recall 0.95
    (deterministic, where the fastest of several such points is noise), and
    the QPS interpolated at 0.95 in (recall, log QPS)."""
    ok = [r for r in curve if r["recall"] >= 0.95]
    best = ok[0] if ok else None
    interp = None
    srt = sorted(curve, key=lambda r: r["recall"])
    for a, b in zip(srt, srt[1:]):
        if a["recall"] < 0.95 <= b["recall"]:
            f = (0.95 - a["recall"]) / (b["recall"] - a["recall"])
            interp = math.exp(math.log(a["qps"]) + f * (math.log(b["qps"]) - math.log(a["qps"])))
    return best, interp


def run_leg(args, cfg: Config, ftype: int, timer, headline: bool):
    """Every mode of one filter type: FP32 fixed, BF16 + rerank fixed, (FP8 +
    rerank fixed on the headline), learned + BF16 + rerank; the operating point
    and its measurements."""
    from paper_2602_10258_amd import jag
    leg = Leg(cfg, ftype, timer)
    log(f"{leg.tag()} {leg.nq} queries")
    fixed = leg.fixed_sweep(cfg.ix32, "fp32")
    fixed16 = leg.fixed_sweep(cfg.ix16, "bf16+rerank", rerank_mult=4)
    L95 = next((r["L"] for r in fixed16 if r["recall"] >= 0.95), None)
    fixed8 = []
    if headline and L95 is not None:
        fixed8 = leg.fixed_sweep(cfg.ix8(), "fp8+rerank", rerank_mult=4,
                                 beams=[L for L in LADDER_FIXED if L95 / 2 <= L <= 2 * L95])
    learned, lad, rep = ([], None, None) if args.only_fixed else leg.learned_sweep(
        args.ntrain, L95, args.ladder_top, args.dump_traces if headline else None)
    # the learned beam over the FP8 store too, where the FP8 fixed beam was swept
    learned8 = [] if args.only_fixed or not fixed8 else leg.learned_sweep(
        args.ntrain, L95, args.ladder_top, None, ix=cfg.ix8(), tag="fp8")[0]
    best_f, interp_f = at95(fixed)
    best_16, interp_16 = at95(fixed16)
    best_8, interp_8 = at95(fixed8) if fixed8 else (None, None)
    best_l, interp_l = at95(learned) if learned else (None, None)
    schedules = None
    if best_l:
        # the sweep runs the two-pass schedule (predict, order by predicted
        # beam, resume); at the chosen offset the one-pass schedule (the
        # prediction taken inside each search, launch order by selectivity
        # class) finds the same ids and may be faster where beams vary little
        one = leg.point(cfg.ix16, jag.SearchParams(L=leg.k, learned=1, delta=best_l["delta"], rerank_mult=4,
                                                   single_pass=1))
        one["delta"] = best_l["delta"]
        schedules = {"two_pass_qps": round(best_l["qps"], 1), "one_pass_qps": round(one["qps"], 1),
                     "one_pass_recall": round(one["recall"], 4)}
        log(f"{leg.tag()} learned at delta={best_l['delta']:g}: two-pass {best_l['qps']:.0f} qps, "
            f"one-pass {one['qps']:.0f} qps (recall {one['recall']:.4f})")
        if one["recall"] >= 0.95 and one["qps"] > best_l["qps"]:
            one["single_pass"] = 1
            best_l = one
    cands = []
    if best_l:
        cands.append(("learned+bf16+rerank" + (" one-pass" if best_l.get("single_pass") else ""), cfg.ix16,
                      jag.SearchParams(L=leg.k, learned=1, delta=best_l["delta"], rerank_mult=4,
                                       single_pass=best_l.get("single_pass", 0)), 1, True, best_l))
    if best_16:
        cands.append(("bf16+rerank-fixed", cfg.ix16, jag.SearchParams(L=best_16["L"], rerank_mult=4), 1, True,
                      best_16))
    if best_f:
        cands.append(("fp32-fixed", cfg.ix32, jag.SearchParams(L=best_f["L"]), 0, False, best_f))
    if best_8:
        cands.append(("fp8+rerank-fixed", cfg.ix8(), jag.SearchParams(L=best_8["L"], rerank_mult=4), 2, True, best_8))
    out = {"workload": f"{FILTER_NAMES[ftype]} filters on {cfg.describe()}", "queries": leg.nq,
           "qps_at_095": {
               "fp32_fixed": best_f and round(best_f["qps"], 1), "fp32_fixed_L": best_f and best_f["L"],
               "fp32_fixed_interp": interp_f and round(interp_f, 1),
               "bf16_rerank_fixed": best_16 and round(best_16["qps"], 1), "bf16_rerank_fixed_L": best_16 and best_16["L"],
               "bf16_rerank_fixed_interp": interp_16 and round(interp_16, 1),
               "fp8_rerank_fixed": best_8 and round(best_8["qps"], 1), "fp8_rerank_fixed_L": best_8 and best_8["L"],
               "learned_fp8_rerank": (at95(learned8)[0] or {}).get("qps") and round(at95(learned8)[0]["qps"], 1),
               "learned_fp8_delta": (at95(learned8)[0] or {}).get("delta"),
               "learned_bf16_rerank": best_l and round(best_l["qps"], 1),
               "learned_bf16_rerank_interp": interp_l and round(interp_l, 1),
               "learned_delta": best_l and best_l["delta"], "learned_mean_beam": best_l and round(best_l["lhat"], 2)},
           "learned_schedules": schedules,
           "learned_target_rule": getattr(leg, "target_rule", None),
           "learned_qps_by_target_rule": getattr(leg, "target_rules", None),
           "learned_over_fp32_fixed": (best_l and best_f and round(best_l["qps"] / best_f["qps"], 4)) or None,
           "learned_over_bf16_fixed": (best_l and best_16 and round(best_l["qps"] / best_16["qps"], 4)) or None,
           "learned_ladder": None if lad is None else lad.tolist(),
           "predictor": rep and rep.__dict__,
           "selectivity_estimate": leg.selectivity_accuracy(),
           "graph_build_seconds": cfg.build_times,
           "sweeps": {"fp32_fixed": [rounded(r) for r in fixed], "bf16_rerank_fixed": [rounded(r) for r in fixed16],
                      "fp8_rerank_fixed": [rounded(r) for r in fixed8], "learned": [rounded(r) for r in learned],
                      "learned_fp8": [rounded(r) for r in learned8]}}
    if not cands:
        top = max(fixed + fixed16 + learned, key=lambda r: r["recall"])
        out["note"] = "no configuration reached recall@10 = 0.95"
        out["best_recall"] = rounded(top)
        return out, None
    # the metric's configuration is the learned beam with the BF16 store; the
    # fastest fixed mode stands in only where the learned search misses 0.95
    op = cands[0] if best_l else max(cands, key=lambda c: c[5]["qps"])
    mode, ix, sp, store, rerank, pt = op
    name = f"{mode} L={sp.L}" if not sp.learned else f"{mode} delta={sp.delta:g}"
    log(f"{leg.tag()} operating point: {name} ({rounded(pt)})")
    out["operating_point"] = name
    out["storage"] = STORE_NAMES[store]
    out.update(leg.op_measure(ix, sp, store, rerank))
    Lcpu = best_f["L"] if best_f else pt.get("L", 64)
    if not args.no_cpu and not headline:
        out["cpu_baseline"] = leg.cpu(Lcpu, args.leg_cpu_seconds, 2000)
    return out, dict(leg=leg, mode=mode, ix=ix, sp=sp, store=store, rerank=rerank, point=pt, name=name, Lcpu=Lcpu)


def predictor_eval(args, dev, timer):
    """Config 4: the predictor trained on 200,000 traces of mixed label, range
    and subset queries over the config-1 data, scored on 10,000 held-out
    queries (mean squared error of the ladder index, and QPS at recall 0.95
    against fixed beams on the same store)."""
    import torch
    from oracle import oracle as O
    from paper_2602_10258_amd import jag
    from paper_2602_10258_amd import predictor as pred
    from workloads import make_config
    from workloads.gen import extra_queries
    t0 = time.time()
    w = make_config("c4", nq=args.c4_heldout)
    thr = [(0, 1.0), (0, 0.01), (0, 0.0), (1, 0.01), (1, 0.0)]
    adj, entry, _ = build_graph(argparse.Namespace(build="device"), w, thr)
    kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    ix32 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_F32, **kw)
    ix16 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_BF16, keep_f32=True, **kw)
    Qt, Ft, pt = extra_queries(w, args.c4_train, qseed=4000)
    lad = pred.LADDER
    P, rho, rep = pred.fit(ix16, Qt, Ft, pt, k=w.k, exact_idx=ix32, rerank_mult=4, ladder=lad)
    log(f"[c4] predictor fitted on {rep.n_train} traces: loss {rep.loss_first:.3f} -> {rep.loss_last:.3f}")

    def score(Q, F, pool):
        Qd, rec = pred._device_batch(ix16, Q, F, pool)
        Qe, rece = pred._device_batch(ix32, Q, F, pool)
        eids, ecnt = pred.exact_answers(ix32, Qe, rece, w.k)
        feats, all_ids, hops = pred.traces(ix16, Qd, rec, w.k, lad, 4)
        tgt, reached = pred.targets_from(all_ids, eids, ecnt, w.k)
        ok = feats[:, 15] == 1.0
        x = feats[ok].astype(np.float64)
        W1, b1 = P[:1024].reshape(64, 16), P[1024:1088]
        W2, b2 = P[1088:5184].reshape(64, 64), P[5184:5248]
        y = np.maximum(np.maximum(x @ W1.T + b1, 0) @ W2.T + b2, 0) @ P[5248:5312] + P[5312]
        t = tgt[ok].astype(np.float64)
        mse = float(np.mean((y - t) ** 2))
        return {"queries": int(ok.sum()), "mse_ladder_index": round(mse, 4),
                "r2": round(1.0 - mse / max(float(np.var(t)), 1e-12), 4),
                "unreachable": int((~reached).sum())}
    train_score = score(Qt[:args.c4_heldout], Ft[:args.c4_heldout], pt)
    held = score(w.Q, w.F, w.pool)
    log(f"[c4] held-out: {held}; training sample: {train_score}")
    # QPS at recall 0.95 on the held-out queries: fixed beams vs the learned beam
    gi, gd, nv = O.bruteforce(w.X, O.attrs_of(w), w.Q, w.F, w.pool, w.k, nthreads=min(os.cpu_count() or 1, 16))
    cfg = argparse.Namespace(name="c4", w=w, gi=gi, nv=nv, dev=dev, torch=torch, ix16=ix16, ix32=ix32)
    out = {"workload": f"c4: mixed label/range/subset queries over the {w.n} x {w.d} config-1 vectors "
                       f"(scalar{{100%,1%,0}}+labels{{1%,0}}), k={w.k}, R={w.R}",
           "train_traces": rep.n_train, "train_loss_first": round(rep.loss_first, 4),
           "train_loss_last": round(rep.loss_last, 4), "heldout": held, "train_sample": train_score}
    legq = {}
    for ft in (0, 1, 2):
        leg = Leg(cfg, ft, timer)
        f32 = leg.fixed_sweep(ix32, "fp32")
        f16 = leg.fixed_sweep(ix16, "bf16+rerank", rerank_mult=4)
        lr = []
        for delta in [-1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]:
            r = leg.point(ix16, jag.SearchParams(L=w.k, learned=1, delta=delta, rerank_mult=4))
            r["delta"] = delta
            lr.append(r)
            if r["recall"] >= 0.95:
                break
        b32, b16, bl = at95(f32)[0], at95(f16)[0], at95(lr)[0]
        one = None
        if bl:  # the one-pass schedule at the same offset (same ids)
            one = leg.point(ix16, jag.SearchParams(L=w.k, learned=1, delta=bl["delta"], rerank_mult=4,
                                                   single_pass=1))
        legq[FILTER_NAMES[ft]] = {
            "learned_one_pass_qps": one and round(one["qps"], 1),
            "fp32_fixed": b32 and {"L": b32["L"], "qps": round(b32["qps"], 1), "expansions": round(b32["hops"], 2)},
            "bf16_rerank_fixed": b16 and {"L": b16["L"], "qps": round(b16["qps"], 1),
                                          "expansions": round(b16["hops"], 2)},
            "learned_bf16_rerank": bl and {"delta": bl["delta"], "qps": round(bl["qps"], 1),
                                           "expansions": round(bl["hops"], 2), "mean_beam": round(bl["lhat"], 2)}}
        log(f"[c4:{FILTER_NAMES[ft]}] {legq[FILTER_NAMES[ft]]}")
    out["heldout_qps_at_095"] = legq
    out["seconds"] = round(time.time() - t0, 1)
    return out


def profile_main(args, dev):
    """Only the operating point of one workload and filter type, for rocprofv3
    (no sweeps, no ground truth)."""
    from paper_2602_10258_amd import jag
    from paper_2602_10258_amd import predictor as pred
    from workloads import make_config
    from workloads.gen import extra_queries
    import torch
    name = args.config or "c2"
    w = make_config(name, n=args.n, nq=args.nq)
    if args.R:
        w = dataclasses.replace(w, R=args.R)
    if args.filter_type is not None:
        keep = w.F[:, 0] == args.filter_type
        w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
    k = w.k
    adj, entry, _ = build_graph(args, w, parse_thresholds(args.thresholds) if args.thresholds else THRESHOLDS[w.name])
    kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    store = {"fp32-fixed": jag.STORE_F32, "bf16+rerank-fixed": jag.STORE_BF16,
             "fp8+rerank-fixed": jag.STORE_FP8_E4M3, "learned+bf16+rerank": jag.STORE_BF16}[args.op_mode]
    ix = jag.jag_build_from_graph(w.X, adj, entry, store=store, keep_f32=store != jag.STORE_F32, **kw)
    if args.op_mode == "learned+bf16+rerank":
        ix32 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_F32, **kw)
        Qt, Ft, pt = extra_queries(w, args.ntrain * (2 if name == "c3" else 1), qseed=1000)
        if args.filter_type is not None:
            keep = Ft[:, 0] == args.filter_type
            Qt, Ft = np.ascontiguousarray(Qt[keep][:args.ntrain]), np.ascontiguousarray(Ft[keep][:args.ntrain])
        lad = (np.array([int(x) for x in args.ladder.split(",")], dtype=np.int32) if args.ladder
               else learned_ladder(None))
        pred.fit(ix, Qt, Ft, pt, k=k, exact_idx=ix32, rerank_mult=4, ladder=lad, unreachable=args.target_rule)
        sp = jag.SearchParams(L=k, learned=1, delta=args.delta, rerank_mult=4,
                              single_pass=1 if args.single_pass else 0)
    else:
        sp = jag.SearchParams(L=args.L, rerank_mult=0 if store == jag.STORE_F32 else 4)
    Qd = torch.from_numpy(w.Q).to(dev)
    rec = torch.from_numpy(jag.jag_encode_filters(ix, w.F, w.pool)).to(dev)
    ids = torch.empty((w.nq, k), dtype=torch.int32, device=dev)
    d2 = torch.empty((w.nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((w.nq,), dtype=torch.int32, device=dev)
    for i in range(args.warmup + args.steps):
        jag.jag_search_encoded(ix, Qd, rec, k, sp, ids, d2, cnt)
    torch.cuda.synchronize()
    log(f"profiled {args.steps} steps of {args.op_mode} L={args.L} on {name} ({w.nq} queries)")
    if args.calib_bytes:
        # a plain device copy of known size, to scale the memory counters
        src = torch.empty(args.calib_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copies of {args.calib_bytes} bytes done")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a layout over several GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve_main(args)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.profile_op:
        return profile_main(args, dev)
    if args.build_only:
        from workloads import make_config
        name = args.config or "c2"
        w = make_config(name, n=args.n, nq=args.nq or 10)
        if args.R:
            w = dataclasses.replace(w, R=args.R)
        thr = parse_thresholds(args.thresholds) if args.thresholds else THRESHOLDS[w.name]
        adj, entry, times = build_graph(args, w, thr)
        print(json.dumps({"workload": w.name, "n": w.n, "d": w.d, "R": w.R, "L_build": 2 * w.R,
                          "thresholds": [list(t) for t in thr], "graph_build_seconds": times,
                          "mean_degree": round(float((adj >= 0).sum(1).mean()), 2)}))
        return
    legs = [tuple(x.split(":")) for x in args.legs.split(",")]
    if args.config:
        legs = [l for l in legs if l[0] == args.config] or [(args.config, t) for t in
                                                              {"c1": ["label"], "c2": ["range"],
                                                               "c3": ["subset", "boolean"], "c4": [],
                                                               "c5": ["label", "range", "subset", "boolean"],
                                                               "bool15": ["table"]}[args.config]]
    timer = Timer()
    configs, results = {}, {}
    headline, serving = {}, None
    t_all = time.time()
    search_legs = [l for l in legs if l[1] != "serve"]
    for i, (cname, tname) in enumerate(legs):
        if cname not in configs:
            # one workload's graph and indexes at a time on the device
            configs.clear()
            types = [FILTER_CODES[t] for c, t in legs if c == cname and t != "serve"]
            configs[cname] = Config(args, cname, dev, types or None)
        if tname == "serve":
            serving = serve_leg(args, configs[cname])
            log(f"leg {tname}:{cname} done at {time.time() - t_all:.0f}s")
            continue
        first = (cname, tname) == search_legs[0]
        out, op = run_leg(args, configs[cname], FILTER_CODES[tname], timer, headline=first)
        results[f"{tname}:{cname}"] = out
        if first:
            headline = timed_steps(args, configs[cname], out, op)
        log(f"leg {tname}:{cname} done at {time.time() - t_all:.0f}s")
    configs.clear()
    c4 = None
    if not args.no_c4 and not args.config:
        c4 = predictor_eval(args, dev, timer)
    if not search_legs:
        print(json.dumps({"metric": "serving latency (p50/p99) and QPS by admission mode", "serving": serving,
                          "seconds": round(time.time() - t_all, 1)}, default=float), flush=True)
        return
    hout = results[f"{search_legs[0][1]}:{search_legs[0][0]}"]
    op = headline.get("op")
    learned_wins = {k_: (v.get("learned_over_bf16_fixed") or 0) > 1.0 for k_, v in results.items()}
    summary = {k_: {"fp32_fixed": v["qps_at_095"]["fp32_fixed"], "bf16_rerank_fixed": v["qps_at_095"]["bf16_rerank_fixed"],
                    "learned_bf16_rerank": v["qps_at_095"]["learned_bf16_rerank"],
                    "learned_over_fp32_fixed": v.get("learned_over_fp32_fixed"),
                    "learned_over_bf16_fixed": v.get("learned_over_bf16_fixed"),
                    "roofline_frac": v.get("roofline", {}).get("frac"), "end_to_end_qps": v.get("end_to_end_qps"),
                    "kernel_qps": v.get("kernel_qps"),
                    **({"fp8_rerank_fixed": v["qps_at_095"]["fp8_rerank_fixed"],
                        "learned_fp8_rerank": v["qps_at_095"]["learned_fp8_rerank"]}
                       if v["qps_at_095"].get("learned_fp8_rerank") else {})} for k_, v in results.items()}
    out = {
        "metric": METRIC, "value": headline.get("value"), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": headline.get("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if op and op["store"] == 1 else "fp8" if op and op["store"] == 2 else "f32",
        "data": "synthetic",
        "config": {"workload": hout["workload"], "filter_type": search_legs[0][1], "global_batch": hout["queries"],
                   "mode": op and op["mode"], "recall_at_10": headline.get("recall"),
                   "storage": op and STORE_NAMES[op["store"]], "accumulate": "fp32"},
        "roofline": hout.get("roofline"),
        "cpu_baseline": hout.get("cpu_baseline"),
        "cpu_baseline_one_thread": headline.get("cpu1"),
        "operating_point": hout.get("operating_point"),
        "kernel_ms": headline.get("kernel_ms"),
        "end_to_end_qps": hout.get("end_to_end_qps"),
        "per_filter_type": summary,
        "learned_beats_bf16_fixed": learned_wins,
        "legs": results,
        "predictor_c4": c4,
        "serving": serving,
        "seconds": round(time.time() - t_all, 1),
    }
    print(json.dumps(out, default=float), flush=True)


def _search_stride(raw: int) -> int:
    """Row stride the search kernels use for rows of `raw` bytes: 64-byte
    padding, then a multiple of 16 bytes per lane of the row's lane group."""
    stride = (raw + 63) // 64 * 64
    g = 4 if stride <= 384 else 8 if stride <= 512 else 16
    return (stride + 16 * g - 1) // (16 * g) * (16 * g)


def gather_ceiling(cfg, leg, st, store, rerank, achieved):
    """The device's rate for reading rows at random, data-dependent indices
    (jag_gather_ceiling, 5,120 waves as the search keeps resident, 4 GiB
    buffer) at the three row sizes of this search -- adjacency rows, store
    rows, FP32 rerank rows -- and the rate the search's algorithmic bytes
    would reach if each of the three streams ran at its row size's rate."""
    from paper_2602_10258_amd import jag
    torch, w = cfg.torch, cfg.w
    info = cfg.ix32.info()
    up4 = lambda x: (x + 3) // 4 * 4  # noqa: E731
    scal = up4(w.R) if info.has_scalar else 0
    lab = up4(scal + w.R if info.has_scalar else w.R) if info.has_labels else 0
    words = up4(lab + w.R * (info.label_width // 2) if info.has_labels else (scal + w.R if info.has_scalar else w.R))
    sizes = {"adjacency": _search_stride(4 * words), "store": _search_stride(row_bytes(w.d, store)),
             "rerank": _search_stride(4 * w.d)}
    # 4 GiB: random rows then rarely hit the 256 MB last-level cache
    buf = torch.empty(1 << 32, dtype=torch.uint8, device=cfg.dev)
    rates = {}
    try:
        for name, b in sizes.items():
            if b not in rates:
                rates[b] = jag.jag_gather_ceiling(buf, b, waves=256 * 20, iters=200, reps=5)
    except jag.JagError as e:
        log(f"gather ceiling not measured: {e}")
        return None
    finally:
        del buf
    parts = {"adjacency": float((st[:, 0] * 4 * w.R + st[:, 2] * attr_bytes(w, leg.ftype)).sum()),
             "store": float((st[:, 1] * row_bytes(w.d, store) + 4 * w.d + 128 + 8 * leg.k + 4).sum()),
             "rerank": float(len(st) * 4 * leg.k * 4 * w.d) if rerank else 0.0}
    total = sum(parts.values())
    mix = total / sum(parts[n] / rates[sizes[n]] for n in parts if parts[n] > 0)
    return {"unit": "GB/s", "row_bytes": sizes, "rate_by_row_bytes": {str(b): round(r, 1) for b, r in rates.items()},
            "mix": round(mix, 1), "frac_of_mix": round(achieved / mix, 4),
            "note": "random rows at data-dependent indices of a 4 GiB buffer, 5,120 one-wave workgroups; the "
                    "mix weighs each row size by the search's algorithmic bytes of that stream"}


def timed_steps(args, cfg, hout, op):
    """The headline leg's operating point: `warmup` untimed steps, then `steps`
    timed ones (HIP events on the search stream, wall clock around all of them),
    the roofline of their kernel time, the committed counters when they match
    this source, and the CPU baseline."""
    import torch
    if op is None:
        return {}
    leg, ix, sp = op["leg"], op["ix"], op["sp"]

    def step():
        leg.search(ix, sp)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    rec = leg.recall(leg.ids.cpu().numpy())
    leg.search(ix, _stats_params(sp, leg.stats))
    torch.cuda.synchronize()
    st = leg.stats.cpu().numpy().astype(np.int64)
    achieved = leg.alg_bytes(st, op["store"], op["rerank"]) / (kern_ms / 1e3) / 1e9
    hout["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(cfg.name, op["name"]),
                        "gather_ceiling": gather_ceiling(cfg, leg, st, op["store"], op["rerank"], achieved)}
    out = {"op": {k_: op[k_] for k_ in ("mode", "store", "rerank", "name")},
           "value": round(leg.nq / (ms_per_step / 1e3), 1), "ms_per_step": round(ms_per_step, 4),
           "kernel_ms": round(kern_ms, 4), "recall": round(rec, 4)}
    if not args.no_cpu:
        from oracle import oracle as O
        hout["cpu_baseline"] = leg.cpu(op["Lcpu"], args.cpu_seconds, args.cpu_sample)
        m1 = max(1, min(args.cpu_sample, leg.nq) // 10)
        t4 = time.time()
        O.search(cfg.w.X, cfg.adj, cfg.entry, cfg.A, leg.Q[:m1], leg.F[:m1], leg.pool, op["Lcpu"], leg.k,
                 nthreads=1)
        out["cpu1"] = {"value": round(m1 / (time.time() - t4), 1), "unit": "queries/s", "cores": 1,
                       "sample": f"first {m1} queries, same beam", "cpu_model": cpu_model()}
    log(f"timed {args.steps} steps: {out['value']:.0f} queries/s, {out['ms_per_step']} ms per step")
    return out


def _stats_params(sp, stats):
    from paper_2602_10258_amd import jag
    return jag.SearchParams(**{**sp.__dict__, "stats": stats})


if __name__ == "__main__":
    main()
