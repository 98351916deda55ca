import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def c1_small():
    """c1 workload (20k x 32, 8 labels) with the oracle-built graph, cached per session."""
    from workloads import make_config
    from oracle import oracle as O
    w = make_config("c1")
    A = O.attrs_of(w)
    import hashlib
    with open(os.path.join(ROOT, "oracle", "jag_oracle.c"), "rb") as f:
        tag = hashlib.sha1(f.read()).hexdigest()[:12]
    cache = os.path.join(ROOT, "tests", f".cache_c1_graph_{tag}.npz")
    if os.path.exists(cache):
        z = np.load(cache)
        adj, entry = z["adj"], int(z["entry"])
    else:
        adj, entry, _ = O.build(w.X, A, 32, 64, 1.2, [O.KIND_LABELS, O.KIND_LABELS], [1.0, 0.0], seed=0)
        np.savez(cache, adj=adj, entry=entry)
    return w, A, adj, entry


import numpy as np  # noqa: E402


@pytest.fixture(scope="session")
def mixed_world():
    """6000 points, d = 24 (a ragged row), a scalar and 1-5 labels per item,
    graph from the oracle builder; 160 queries of all four filter types."""
    from oracle import oracle as O
    from workloads import (FILTER_LABEL, FILTER_RANGE, FILTER_SUBSET, Workload, encode_filters,
                           make_config)
    rng = np.random.default_rng(21)
    w = make_config("c4", n=6000, nq=4)
    X = (w.X[:, :24] + rng.normal(0, 0.1, size=(6000, 24))).astype(np.float32)
    sets = [sorted(rng.choice(20, size=rng.integers(1, 6), replace=False).tolist()) for _ in range(6000)]
    loff = np.zeros(6001, dtype=np.int64)
    loff[1:] = np.cumsum([len(s) for s in sets])
    lab = np.array([v for s in sets for v in s], dtype=np.int32)
    scal = rng.integers(0, 10000, size=6000).astype(np.int32)
    kinds, pays = [], []
    for i in range(160):
        t = i % 4
        kinds.append(t)
        if t == FILTER_LABEL:
            pays.append(int(rng.integers(0, 20)))
        elif t == FILTER_RANGE:
            lo = int(rng.integers(0, 10000))
            pays.append((lo, lo + int(10 ** rng.uniform(0, 4))))
        elif t == FILTER_SUBSET:
            pays.append(sorted(rng.choice(20, size=rng.integers(1, 4), replace=False).tolist()))
        else:
            a, b, c = rng.choice(20, size=3, replace=False).tolist()
            pays.append([[a, b], [c]] if i % 8 == 3 else [[a, ~b], [c, b]])
    F, pool = encode_filters(kinds, pays)
    Q = (X[rng.integers(0, 6000, size=160)] + rng.normal(0, 0.5, size=(160, 24))).astype(np.float32)
    ww = Workload("mixed", X, Q, F, pool, scal, loff, lab, 20, k=10, R=24, L=64)
    A = O.attrs_of(ww)
    adj, entry, _ = O.build(X, A, 24, 48, 1.2, [O.KIND_SCALAR] * 3 + [O.KIND_LABELS],
                            [1.0, 0.01, 0.0, 0.0], seed=5)
    return ww, A, adj, entry
