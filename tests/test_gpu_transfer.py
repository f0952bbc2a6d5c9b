"""Host <-> device transfer measurement (the paper's transfer figure, Section
5.2, which prints no numbers): pinned and pageable host buffers, both
directions, timed with events, energy from the GPU counter when present.
The data must arrive intact and the rates be positive; pinned H2D / D2H are
not slower than a tenth of pageable (the usual order is the reverse)."""
import numpy as np
import pytest
import torch

import bench

pytestmark = pytest.mark.gpu


def test_round_trip_intact():
    n = (8 << 20) // 8
    src = torch.from_numpy(np.arange(n, dtype=np.float64) * 0.5 - 3.0)
    for pinned in (True, False):
        h = src.pin_memory() if pinned else src.clone()
        d = torch.empty(n, dtype=torch.float64, device="cuda")
        d.copy_(h, non_blocking=pinned)
        back = torch.empty(n, dtype=torch.float64, pin_memory=pinned)
        back.copy_(d, non_blocking=pinned)
        torch.cuda.synchronize()
        assert torch.equal(back, src)


def test_transfer_rows():
    meter = bench.EnergyMeter()
    res = bench.extra_transfer(meter, sizes_mib=(4,), min_s=1.0)
    rows = res["rows"]
    assert len(rows) == 4
    for r in rows:
        assert r["GBs"] > 0.5, r
        if meter.sampler.ok and r["j_per_GB"] is not None:
            assert 0.0 < r["j_per_GB"] < 1000.0, r
    by = {(r["pinned"], r["dir"]): r["GBs"] for r in rows}
    for d in ("h2d", "d2h"):
        assert by[(True, d)] > 0.1 * by[(False, d)]
