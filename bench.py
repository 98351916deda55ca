"""Benchmark: filtered QPS at recall@10 = 0.95 on one MI355X.

Default workload (range filters, the study's headline shape): 1,000,000
vectors, d = 96, 256-cluster Gaussian mixture, one int32 attribute uniform
over [0, 10^6); 10,000 range queries with log-uniform selectivity over
[1e-4, 1]; k = 10; graph R = 64, thresholds {100%, 1%, 0} of the scalar.

Setup (untimed): build the Threshold-JAG (on the GPU by default; --build
host or both), lay out FP32, BF16 and FP8 indexes (with FP32 copies) over
the same graph, compute the exact answers with the CPU oracle (FP64), sweep
the fixed beam L for each store, fit the beam predictor on a separate query
set (GPU kernels), sweep its offset for learned + BF16 + FP32-rerank search.
Each mode's point is the smallest sweep beam or offset reaching recall
>= 0.95 (grid points, then bisection between the bracketing ones); the
timed steps run the learned + BF16 point over the whole query batch
(the fastest fixed mode where the learned search misses 0.95), inputs
resident in HBM.  One JSON line on stdout.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config c2|c1|c3|c5|bool15]
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
    ap.add_argument("--config", default="c2")
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
    ap.add_argument("--ladder", default=None,
                    help="profile mode, learned: comma-separated ladder (as the bench line reports it)")
    ap.add_argument("--ladder-top", type=int, default=None,
                    help="widest beam of the learned ladder (default: 1.4x the fixed beam at recall 0.95)")
    ap.add_argument("--dump-traces", default=None, help="save predictor traces to this .npz")
    ap.add_argument("--serve", action="store_true", help="serving benchmark (Poisson arrivals)")
    ap.add_argument("--rates", default="5000,20000,50000,100000,200000")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="profile mode: also run device copies of this many bytes")
    ap.add_argument("--min-valid", type=int, default=None,
                    help="drop queries with fewer valid items (default: k for the label-set "
                         "workloads c3 and c5, else 0)")
    ap.add_argument("--filter-type", type=int, default=None, choices=[0, 1, 2, 3, 4],
                    help="keep only the queries of this filter type (0 label, 1 range, 2 subset, 3 Boolean)")
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


def measured_traffic(workload: str, op_name: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summaries (one entry, or a list of entries, one per operating point),
    only if taken on this exact kernel source and operating point;
    otherwise None."""
    import hashlib
    p = os.path.join(ROOT, "profiles", f"search_kernel_{workload}_counters.json")
    src = os.path.join(ROOT, "paper_2602_10258_amd", "csrc", "search.hip")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for e in d if isinstance(d, list) else [d]:
        if e.get("search_hip_sha1") == sha and e.get("operating_point") == op_name:
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
    for qps in rates:
        m = min(w.nq, max(2000, int(qps * 1.0)))
        arr = poisson_arrivals(np.random.default_rng(int(qps)), m, qps)
        s = jag.jag_server_start(ix, k, sp, max_batch=4096, n_streams=4, max_wait_us=100)
        t0 = time.perf_counter()
        tick = np.empty(m, dtype=np.uint64)
        i = 0
        while i < m:
            now = time.perf_counter() - t0
            j = int(np.searchsorted(arr, now, side="right"))
            if j > i:
                tick[i:j] = jag.jag_server_submit(s, w.Q[i:j], w.F[i:j], w.pool)
                i = j
            else:
                time.sleep(max(0.0, min(1e-4, arr[i] - now)))
        jag.jag_server_drain(s)
        st = jag.jag_server_stats_get(s)
        got = np.empty((m, k), dtype=np.int32)
        for q in range(m):
            got[q] = jag.jag_server_poll(s, int(tick[q]))[0]
        jag.jag_server_stop(s)
        r = recall_of(got)
        row = {"offered_qps": qps, "requests": m, "achieved_qps": round(st["qps"], 1),
               "p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
               "mean_batch": round(st["mean_batch"], 1), "max_inflight": st["max_inflight_seen"],
               "resident_capacity": st["resident_capacity"], "recall_at_10": round(r, 4)}
        log(row)
        per_rate.append(row)
    out = {"metric": "serving latency (p50/p99) and QPS, mixed filters, learned beam + FP8 + FP32 rerank",
           "config": {"workload": f"c5 shard: {w.n} x {w.d} (10M / 8), FP8 E4M3 + per-row scale, "
                                  f"R={w.R}, mixed Label/Range/Subset/Boolean, Poisson arrivals",
                      "delta": delta, "rho": rho},
           "rates": per_rate}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a layout over several GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve_main(args)
    import torch
    from paper_2602_10258_amd import jag
    from paper_2602_10258_amd import predictor as pred
    from workloads import make_config
    from workloads.gen import extra_queries

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = make_config(args.config, n=args.n, nq=args.nq)
    if args.R:
        w = dataclasses.replace(w, R=args.R)
    if args.filter_type is not None:
        keep = w.F[:, 0] == args.filter_type
        assert keep.any(), f"no queries of filter type {args.filter_type} in {w.name}"
        w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
    k = w.k
    log(f"workload {w.name}: n={w.n} d={w.d} nq={w.nq} ({time.time() - t0:.1f}s)")

    # ---- build the graph and lay out the two stores over it
    thr_list = parse_thresholds(args.thresholds) if args.thresholds else THRESHOLDS[w.name]
    t1 = time.time()
    if args.graph_cache and os.path.exists(args.graph_cache):
        z = np.load(args.graph_cache)
        adj, entry = z["adj"], int(z["entry"])
        build_times = {"cached": 0.0}
        log(f"graph loaded from {args.graph_cache}")
    else:
        adj, entry, build_times = build_graph(args, w, thr_list)
        if args.graph_cache:
            np.savez(args.graph_cache, adj=adj, entry=entry)
    build_s = time.time() - t1
    log(f"graph built in {build_s:.1f}s, mean degree {(adj >= 0).sum(1).mean():.1f}")
    if args.build_only:
        print(json.dumps({"workload": w.name, "n": w.n, "d": w.d, "R": w.R, "L_build": 2 * w.R,
                          "thresholds": [list(t) for t in thr_list],
                          "graph_build_seconds": build_times,
                          "mean_degree": round(float((adj >= 0).sum(1).mean()), 2)}))
        return
    kw = dict(scalar=w.scalar, label_off=w.loff, labels=w.lab, vocab=w.vocab)
    ix32 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_F32, **kw)
    ix16 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_BF16, keep_f32=True, **kw)
    rec32 = torch.from_numpy(jag.jag_encode_filters(ix32, w.F, w.pool)).to(dev)
    rec16 = torch.from_numpy(jag.jag_encode_filters(ix16, w.F, w.pool)).to(dev)
    Qd = torch.from_numpy(w.Q).to(dev)
    nq = w.nq
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    d2 = torch.empty((nq, k), dtype=torch.float32, device=dev)
    cnt = torch.empty((nq,), dtype=torch.int32, device=dev)
    stats = torch.zeros((nq, 4), dtype=torch.int32, device=dev)

    if args.profile_op:
        # only the operating point, for rocprofv3 (no sweeps, no ground truth)
        if args.op_mode == "fp32-fixed":
            ix, rec, sp = ix32, rec32, jag.SearchParams(L=args.L)
        elif args.op_mode == "bf16+rerank-fixed":
            ix, rec, sp = ix16, rec16, jag.SearchParams(L=args.L, rerank_mult=4)
        elif args.op_mode == "fp8+rerank-fixed":
            ix = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_FP8_E4M3, keep_f32=True, **kw)
            rec = torch.from_numpy(jag.jag_encode_filters(ix, w.F, w.pool)).to(dev)
            sp = jag.SearchParams(L=args.L, rerank_mult=4)
        else:
            Qt, Ft, pt = extra_queries(w, args.ntrain, qseed=1000)
            lad = (np.array([int(x) for x in args.ladder.split(",")], dtype=np.int32) if args.ladder
                   else learned_ladder(None))
            pred.fit(ix16, Qt, Ft, pt, k=k, exact_idx=ix32, rerank_mult=4, ladder=lad)
            ix, rec, sp = ix16, rec16, jag.SearchParams(L=k, learned=1, delta=args.delta, rerank_mult=4)
        for i in range(args.warmup + args.steps):
            jag.jag_search_encoded(ix, Qd, rec, k, sp, ids, d2, cnt)
        torch.cuda.synchronize()
        log(f"profiled {args.steps} steps of {args.op_mode} L={args.L}")
        if args.calib_bytes:
            # a plain device copy of known size, to scale the memory counters
            src = torch.empty(args.calib_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"calibration copies of {args.calib_bytes} bytes done")
        return

    # ---- ground truth: the oracle's exact filtered k-NN in FP64
    from oracle import oracle as O
    t2 = time.time()
    nthr = min(os.cpu_count() or 1, 16)
    A = O.attrs_of(w)
    gi, gd, nv = O.bruteforce(w.X, A, w.Q, w.F, w.pool, k, nthreads=nthr)
    log(f"exact answers (oracle, {nthr} threads) in {time.time() - t2:.1f}s")
    min_valid = args.min_valid if args.min_valid is not None else (k if w.name in ("c3", "c5") else 0)
    if min_valid > 0 and (nv < min_valid).any():
        # label-set workloads keep only queries with at least k valid items
        keep = nv >= min_valid
        log(f"keeping {int(keep.sum())} of {len(keep)} queries with >= {min_valid} valid items")
        w = dataclasses.replace(w, Q=np.ascontiguousarray(w.Q[keep]), F=np.ascontiguousarray(w.F[keep]))
        gi, gd, nv = gi[keep], gd[keep], nv[keep]
        rec32 = torch.from_numpy(jag.jag_encode_filters(ix32, w.F, w.pool)).to(dev)
        rec16 = torch.from_numpy(jag.jag_encode_filters(ix16, w.F, w.pool)).to(dev)
        Qd = torch.from_numpy(w.Q).to(dev)
        nq = w.nq
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        d2 = torch.empty((nq, k), dtype=torch.float32, device=dev)
        cnt = torch.empty((nq,), dtype=torch.int32, device=dev)
        stats = torch.zeros((nq, 4), dtype=torch.int32, device=dev)
    has_valid = nv > 0

    def recall(ids_np):
        hits = np.zeros(nq)
        for q in range(nq):
            den = min(k, int(nv[q]))
            if den:
                hits[q] = len(set(gi[q, :den].tolist()) & set(ids_np[q].tolist())) / den
        return float(hits[has_valid].mean())

    timer = Timer()

    def point(ix, rec, sp):
        def fn():
            jag.jag_search_encoded(ix, Qd, rec, k, sp, ids, d2, cnt)
        ms = timer.run(fn, reps=7, warm=1)
        sp2 = jag.SearchParams(**{**sp.__dict__, "stats": stats})
        jag.jag_search_encoded(ix, Qd, rec, k, sp2, ids, d2, cnt)
        torch.cuda.synchronize()
        st = stats.cpu().numpy()
        return dict(ms=ms, qps=nq / (ms / 1e3), recall=recall(ids.cpu().numpy()),
                    hops=float(st[:, 0].mean()), ndist=float(st[:, 1].mean()),
                    nattr=float(st[:, 2].mean()), lhat=float(st[:, 3].mean()))

    def refine_fixed(curve, run):
        # bisect the integer beams between the last grid point below recall
        # 0.95 and the first at or above it, so that the measured point is
        # the smallest beam reaching 0.95, not the next grid beam
        j = next((i for i, r in enumerate(curve) if r["recall"] >= 0.95), None)
        if not j:
            return
        lo, hi = curve[j - 1]["L"], curve[j]["L"]
        while hi - lo > 1:
            mid = (lo + hi) // 2
            r = run(mid)
            r["L"] = mid
            curve.append(r)
            log(f"  refine L={mid:4d} recall={r['recall']:.4f} qps={r['qps']:.0f}")
            lo, hi = (lo, mid) if r["recall"] >= 0.95 else (mid, hi)
        curve.sort(key=lambda r: r["L"])

    # ---- plain FP32, fixed beam sweep
    ladder_fixed = LADDER_FIXED
    fixed = []
    for L in ladder_fixed:
        r = point(ix32, rec32, jag.SearchParams(L=L))
        r["L"] = L
        fixed.append(r)
        log(f"fp32 L={L:4d} recall={r['recall']:.4f} qps={r['qps']:.0f} hops={r['hops']:.1f}")
        if r["recall"] >= 0.99:
            break
    refine_fixed(fixed, lambda L: point(ix32, rec32, jag.SearchParams(L=L)))
    # ---- ablation: BF16 + FP32 rerank with a fixed beam (no predictor)
    fixed16 = []
    for L in ladder_fixed:
        r = point(ix16, rec16, jag.SearchParams(L=L, rerank_mult=4))
        r["L"] = L
        fixed16.append(r)
        log(f"bf16+rerank L={L:4d} recall={r['recall']:.4f} qps={r['qps']:.0f}")
        if r["recall"] >= 0.99:
            break
    refine_fixed(fixed16, lambda L: point(ix16, rec16, jag.SearchParams(L=L, rerank_mult=4)))
    # ---- ablation: FP8 E4M3 (per-row scale) + FP32 rerank, beams around BF16's 0.95 point
    fixed8 = []
    L95 = next((r["L"] for r in fixed16 if r["recall"] >= 0.95), None)
    if L95 is not None and not args.only_fixed:
        ix8 = jag.jag_build_from_graph(w.X, adj, entry, store=jag.STORE_FP8_E4M3, keep_f32=True, **kw)
        rec8 = torch.from_numpy(jag.jag_encode_filters(ix8, w.F, w.pool)).to(dev)
        for L in [L for L in ladder_fixed if L95 / 2 <= L <= 2 * L95]:
            r = point(ix8, rec8, jag.SearchParams(L=L, rerank_mult=4))
            r["L"] = L
            fixed8.append(r)
            log(f"fp8+rerank L={L:4d} recall={r['recall']:.4f} qps={r['qps']:.0f}")
        refine_fixed(fixed8, lambda L: point(ix8, rec8, jag.SearchParams(L=L, rerank_mult=4)))

    # ---- learned + BF16 + FP32 rerank
    learned = []
    fit_rep = None
    lad = None
    if not args.only_fixed:
        t3 = time.time()
        Qt, Ft, pt = extra_queries(w, args.ntrain, qseed=1000)
        L95 = next((r["L"] for r in fixed16 if r["recall"] >= 0.95), None)
        for top in ladder_tops(L95, args.ladder_top):
            lad = learned_ladder(L95, top)
            log(f"learned ladder {lad.tolist()}")
            P, rho, fit_rep = pred.fit(ix16, Qt, Ft, pt, k=k, exact_idx=ix32, rerank_mult=4,
                                       dump=args.dump_traces, ladder=lad)
            log(f"predictor fitted on {fit_rep.n_train} traces in {time.time() - t3:.1f}s: loss "
                f"{fit_rep.loss_first:.3f} -> {fit_rep.loss_last:.3f}, rho={rho:.2f}, "
                f"unreachable={fit_rep.unreachable}")
            learned = []
            for delta in [-1.0, -0.5, 0.0, 0.5, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 4.0]:
                r = point(ix16, rec16, jag.SearchParams(L=k, learned=1, delta=delta, rerank_mult=4))
                r["delta"] = delta
                learned.append(r)
                log(f"learned+bf16 delta={delta:+.2f} recall={r['recall']:.4f} qps={r['qps']:.0f} "
                    f"mean Lhat={r['lhat']:.1f}")
                if r["recall"] >= 0.995:
                    break
            if any(r["recall"] >= 0.95 for r in learned):
                break
        # bisect the offset between the last sweep point below 0.95 and the
        # first at or above it (four halvings of the grid step; midpoints
        # rounded to 4 decimals, as the report and the profiles name them)
        j = next((i for i, r in enumerate(learned) if r["recall"] >= 0.95), None)
        if j:
            lo, hi = learned[j - 1]["delta"], learned[j]["delta"]
            for _ in range(4):
                mid = round((lo + hi) / 2, 4)
                r = point(ix16, rec16, jag.SearchParams(L=k, learned=1, delta=mid, rerank_mult=4))
                r["delta"] = mid
                learned.append(r)
                log(f"  refine delta={mid:+.4f} recall={r['recall']:.4f} qps={r['qps']:.0f}")
                lo, hi = (lo, mid) if r["recall"] >= 0.95 else (mid, hi)
            learned.sort(key=lambda r: r["delta"])

    def at95(curve):
        # the first sweep point (smallest beam or offset) at or above 0.95:
        # deterministic, where the fastest of several such points is noise
        ok = [r for r in curve if r["recall"] >= 0.95]
        best = ok[0] if ok else None
        interp = None
        srt = sorted(curve, key=lambda r: r["recall"])
        for a, b in zip(srt, srt[1:]):
            if a["recall"] < 0.95 <= b["recall"]:
                f = (0.95 - a["recall"]) / (b["recall"] - a["recall"])
                interp = math.exp(math.log(a["qps"]) + f * (math.log(b["qps"]) - math.log(a["qps"])))
        return best, interp

    best_f, interp_f = at95(fixed)
    best_f16, interp_f16 = at95(fixed16)
    best_f8, interp_f8 = at95(fixed8) if fixed8 else (None, None)
    best_l, interp_l = at95(learned) if learned else (None, None)
    cands = []
    if best_l:
        cands.append(dict(mode="learned+bf16+rerank", ix=ix16, rec=rec16,
                          sp=jag.SearchParams(L=k, learned=1, delta=best_l["delta"], rerank_mult=4),
                          store=jag.STORE_BF16, rerank=True, point=best_l))
    if best_f16:
        cands.append(dict(mode="bf16+rerank-fixed", ix=ix16, rec=rec16,
                          sp=jag.SearchParams(L=best_f16["L"], rerank_mult=4),
                          store=jag.STORE_BF16, rerank=True, point=best_f16))
    if best_f:
        cands.append(dict(mode="fp32-fixed", ix=ix32, rec=rec32, sp=jag.SearchParams(L=best_f["L"]),
                          store=jag.STORE_F32, rerank=False, point=best_f))
    if best_f8:
        cands.append(dict(mode="fp8+rerank-fixed", ix=ix8, rec=rec8,
                          sp=jag.SearchParams(L=best_f8["L"], rerank_mult=4),
                          store=jag.STORE_FP8_E4M3, rerank=True, point=best_f8))
    if not cands:
        # nothing reaches the target: report the sweeps and the best recall seen
        allp = [dict(r, mode=m) for m, rs in (("fp32-fixed", fixed), ("bf16+rerank-fixed", fixed16),
                                              ("fp8+rerank-fixed", fixed8), ("learned+bf16+rerank", learned))
                for r in rs]
        top = max(allp, key=lambda r: r["recall"])
        print(json.dumps({
            "metric": METRIC, "value": None, "unit": "queries/s", "n_gpus": 1, "steps": 0,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{w.name}: {w.n} x {w.d} clustered vectors, {nq} queries "
                                   f"({args.thresholds or w.meta.get('thresholds')}), k={k}, R={w.R}",
                       "global_batch": nq, "filter_types": sorted({FILTER_NAMES[int(t)] for t in w.F[:, 0]})},
            "note": "no configuration reached recall@10 = 0.95",
            "best_recall": {k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in top.items()},
            "graph_build_seconds": build_times,
            "sweeps": {"fixed": fixed, "bf16_rerank_fixed": fixed16, "fp8_rerank_fixed": fixed8,
                       "learned": learned}}, default=float))
        return
    # the metric's configuration is the learned beam with the BF16 store;
    # the fastest fixed-beam mode stands in only where it misses 0.95
    op = cands[0] if best_l else max(cands, key=lambda c: c["point"]["qps"])
    log(f"operating point: {op['mode']} ({op['point']})")

    # ---- timed steps
    def step():
        jag.jag_search_encoded(op["ix"], Qd, op["rec"], k, op["sp"], ids, d2, cnt)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t_start = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / args.steps
    value = nq / (ms_per_step / 1e3)
    rec_final = recall(ids.cpu().numpy())

    # end to end from host filters: encoding, record upload and search
    # (jag_search_batch), query vectors and outputs already on the device
    def step_host():
        jag.jag_search_batch(op["ix"], Qd, w.F, w.pool, k, op["sp"], ids, d2, cnt)
    step_host()
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    for _ in range(args.steps):
        step_host()
    torch.cuda.synchronize()
    e2e_qps = nq * args.steps / (time.perf_counter() - t_h)

    # ---- roofline: algorithmic bytes of one launch / its average duration
    sp2 = jag.SearchParams(**{**op["sp"].__dict__, "stats": stats})
    jag.jag_search_encoded(op["ix"], Qd, op["rec"], k, sp2, ids, d2, cnt)
    torch.cuda.synchronize()
    st = stats.cpu().numpy().astype(np.int64)
    info = op["ix"].info()
    row = w.d * {0: 4, 1: 2, 2: 1}[op["store"]] + (4 if op["store"] == 2 else 0)
    attr = 4 if w.name == "c2" else 2 * max(1, info.label_width)
    per_q = st[:, 0] * 4 * w.R + st[:, 2] * attr + st[:, 1] * row + 4 * w.d + 128 + 8 * k + 4
    if op["rerank"]:
        per_q = per_q + 4 * k * 4 * w.d
    alg_bytes = float(per_q.sum())
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    op_name = (f"{op['mode']} L={op['sp'].L}" if not op["sp"].learned
               else f"{op['mode']} delta={op['sp'].delta:g}")
    traffic = measured_traffic(w.name, op_name)

    # ---- CPU baseline: the oracle, unchanged, on a bounded sample at the same beam
    cpu = cpu1 = None
    if not args.no_cpu:
        m = min(args.cpu_sample, nq)
        Lcpu = op["point"].get("L", best_f["L"] if best_f else 64)
        reps, cs = 0, 0.0
        while reps == 0 or cs < args.cpu_seconds:  # whole passes over the sample, about cpu_seconds
            t4 = time.time()
            O.search(w.X, adj, entry, A, w.Q[:m], w.F[:m], w.pool, Lcpu, k, nthreads=nthr)
            cs += time.time() - t4
            reps += 1
        cpu = {"value": reps * m / cs, "unit": "queries/s", "cores": nthr, "kind": "oracle",
               "sample": f"first {m} of the {nq} queries, {reps} passes, plain FP32 fixed beam L={Lcpu}, "
                         f"FP64 distances, {cs:.1f}s"}
        # the same on one thread, over a tenth of the sample
        m1 = max(1, m // 10)
        t4 = time.time()
        O.search(w.X, adj, entry, A, w.Q[:m1], w.F[:m1], w.pool, Lcpu, k, nthreads=1)
        cpu1 = {"value": round(m1 / (time.time() - t4), 1), "unit": "queries/s", "cores": 1,
                "sample": f"first {m1} queries, same beam", "cpu_model": cpu_model()}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} x {w.d} clustered vectors, {nq} queries "
                               f"({args.thresholds or w.meta.get('thresholds')}), k={k}, R={w.R}",
                   "global_batch": nq, "mode": op["mode"], "recall_at_10": round(rec_final, 4),
                   "filter_types": sorted({FILTER_NAMES[int(t)] for t in w.F[:, 0]}),
                   "storage": {jag.STORE_F32: "fp32", jag.STORE_BF16: "bf16 (+fp32 rerank)",
                               jag.STORE_FP8_E4M3: "fp8 e4m3 + row scale (+fp32 rerank)"}[op["store"]]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic},
        "operating_point": op_name,
        "learned_ladder": None if lad is None else lad.tolist(),
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu1,
        "qps_at_095": {
            "learned_bf16_measured": best_l and round(best_l["qps"], 1),
            "learned_bf16_interp": interp_l and round(interp_l, 1),
            "fp32_fixed_measured": best_f and round(best_f["qps"], 1),
            "fp32_fixed_interp": interp_f and round(interp_f, 1),
            "fp32_fixed_L": best_f and best_f["L"],
            "bf16_rerank_fixed_measured": best_f16 and round(best_f16["qps"], 1),
            "bf16_rerank_fixed_interp": interp_f16 and round(interp_f16, 1),
            "bf16_rerank_fixed_L": best_f16 and best_f16["L"],
            "fp8_rerank_fixed_measured": best_f8 and round(best_f8["qps"], 1),
            "fp8_rerank_fixed_interp": interp_f8 and round(interp_f8, 1),
            "fp8_rerank_fixed_L": best_f8 and best_f8["L"],
        },
        "kernel_ms": round(kern_ms, 4),
        "host_filters_qps": round(e2e_qps, 1),
        "alg_bytes_per_query": round(alg_bytes / nq, 1),
        "mean_expansions": round(float(st[:, 0].mean()), 2),
        "mean_distance_computations": round(float(st[:, 1].mean()), 2),
        "build_seconds": round(build_s, 1),
        "graph_build_seconds": build_times,
        "sweeps": {"fixed": [{k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in r.items()}
                             for r in fixed],
                   "bf16_rerank_fixed": [{k_: (round(v, 4) if isinstance(v, float) else v)
                                          for k_, v in r.items()} for r in fixed16],
                   "fp8_rerank_fixed": [{k_: (round(v, 4) if isinstance(v, float) else v)
                                         for k_, v in r.items()} for r in fixed8],
                   "learned": [{k_: (round(v, 4) if isinstance(v, float) else v) for k_, v in r.items()}
                               for r in learned]},
        "predictor": fit_rep and fit_rep.__dict__,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
