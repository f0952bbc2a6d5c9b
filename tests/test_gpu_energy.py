"""The energy measurement on the GPU (the paper's Section 4 protocol, with the
GPU's own energy counter in place of clamps and an oscilloscope): the
background sampler sees the counter advance, a window's mean power lies in
the board's range, a load phase between two idle phases reads higher than
both, and the phase analysis (averaging filter, step detection on the
variance with a noise sample, short boundary segments folded back) recovers
the idle / load / idle pattern from the sampled trace."""
import time

import numpy as np
import pytest
import torch

from paper_2112_10823_amd import cgx
from paper_2112_10823_amd.energy import (EnergySampler, detect_steps, merge_short,
                                         moving_average, noise_from_differences, phase_pattern,
                                         segments_of)

pytestmark = pytest.mark.gpu


def test_sampler_and_phase_analysis_on_an_idle_load_idle_run():
    s = EnergySampler(period_s=0.005)
    if not s.ok:
        pytest.skip("no amdsmi energy counter on this machine")
    n = 1 << 25
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.rand(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(x)
    h = cgx.default_handle()
    with s:
        t0 = time.perf_counter()
        time.sleep(4.0)                       # idle
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < 5.0:  # load: back-to-back vector additions
            for _ in range(50):
                cgx.add(x, y, z, handle=h)
            torch.cuda.synchronize()
        t2 = time.perf_counter()
        time.sleep(4.0)                       # idle
        t3 = time.perf_counter()
    assert len(s.updates) >= 8, len(s.updates)
    p_idle0 = s.power_between(t0 + 1.0, t1)
    p_load = s.power_between(t1 + 1.5, t2)
    p_idle1 = s.power_between(t2 + 1.5, t3)
    assert None not in (p_idle0, p_load, p_idle1)
    for p in (p_idle0, p_load, p_idle1):
        assert 20.0 < p < 2500.0
    assert p_load > max(p_idle0, p_idle1) + 50.0, (p_idle0, p_load, p_idle1)
    # the paper's analysis on the trace: filter, steps, boundary samples folded back
    tt, pw = s.trace()
    keep = (tt >= t0) & (tt <= t3)
    tr = moving_average(pw[keep], 1)
    sigma = max(noise_from_differences(tr), 10.0)
    cuts = merge_short(tr, detect_steps(tr, sigma), 2)
    segs = segments_of(tr, cuts)
    pat = phase_pattern(segs)
    assert pat[0] >= 3 and 1 in pat[1:] and -1 in pat[1:], (pat, [sg.level for sg in segs])
    top = max(segs, key=lambda sg: sg.level)
    assert abs(top.level - p_load) <= 0.25 * p_load
