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
