"""GPU test of the random row-gather probe that the benchmark prices the
search's memory streams with."""
import pytest

from paper_2602_10258_amd import jag

pytestmark = pytest.mark.gpu


def test_gather_ceiling_rates_are_plausible():
    import torch
    buf = torch.zeros(1 << 28, dtype=torch.uint8, device="cuda")
    r192 = jag.jag_gather_ceiling(buf, 192, waves=2048, iters=50, reps=2)
    r512 = jag.jag_gather_ceiling(buf, 512, waves=2048, iters=50, reps=2)
    print("[gpu] gather GB/s: 192 B rows", round(r192), "512 B rows", round(r512), flush=True)
    # random rows cannot beat the 8 TB/s peak (no row is read twice on purpose;
    # the 256 MiB buffer fits the 256 MB last-level cache only in part)
    assert 100 < r192 < 12000 and 100 < r512 < 12000
