"""CPU tests of the power-trace analysis (the paper's Section 4: averaging
filter, variance-based step detection given a noise sample, most common
phase pattern over repeated runs) on synthetic traces whose phases are
known."""
import numpy as np
import pytest

from paper_2112_10823_amd.energy import (detect_steps, merge_short, most_common_pattern,
                                         moving_average, noise_from_differences, phase_pattern,
                                         robust_spread, segments_of)

LEVELS = [250.0, 800.0, 600.0, 820.0, 260.0]
LENGTHS = [8, 10, 6, 12, 9]


def synthetic(seed, sigma=5.0, levels=LEVELS, lengths=LENGTHS):
    rng = np.random.default_rng(seed)
    truth = np.concatenate([np.full(n, v) for v, n in zip(levels, lengths)])
    return truth + rng.normal(0.0, sigma, truth.size), list(np.cumsum(lengths)[:-1])


def test_moving_average_definition():
    rng = np.random.default_rng(0)
    x = rng.normal(size=37)
    for w in (1, 3, 5, 9):
        y = moving_average(x, w)
        h = w // 2
        ref = [x[max(0, i - h):i + h + 1].mean() for i in range(x.size)]
        assert np.allclose(y, ref, rtol=0, atol=1e-12)
    assert np.array_equal(moving_average(np.full(10, 3.5), 5), np.full(10, 3.5))


@pytest.mark.parametrize("seed", range(6))
def test_steps_recovered_exactly(seed):
    x, cuts = synthetic(seed)
    found = detect_steps(x, noise_std=5.0, min_len=2)
    assert found == cuts
    for s, v, n in zip(segments_of(x, found), LEVELS, LENGTHS):
        assert abs(s.level - v) <= 4 * 5.0 / np.sqrt(n)


@pytest.mark.parametrize("seed", range(8))
def test_noise_alone_has_no_step(seed):
    rng = np.random.default_rng(100 + seed)
    x = 400.0 + rng.normal(0.0, 5.0, 60)
    assert detect_steps(x, noise_std=5.0) == []


def test_underestimated_noise_gives_spurious_steps():
    """The noise sample matters: told the noise is ten times smaller than it
    is, the detector cuts the noise itself."""
    rng = np.random.default_rng(7)
    x = 400.0 + rng.normal(0.0, 5.0, 60)
    assert len(detect_steps(x, noise_std=0.5)) > 0


def test_min_len_and_single_step_at_the_edge():
    x = np.concatenate([np.full(3, 100.0), np.full(30, 500.0)])
    assert detect_steps(x, noise_std=1.0, min_len=2) == [3]
    assert detect_steps(x, noise_std=1.0, min_len=4) in ([4], [])


def test_most_common_pattern_average():
    a = [(2.0, 250.0), (5.0, 800.0), (3.0, 260.0)]
    b = [(2.2, 254.0), (4.8, 790.0), (3.1, 262.0)]
    odd = [(2.0, 250.0), (1.0, 600.0), (4.0, 800.0), (3.0, 255.0)]
    pat, keep, phases = most_common_pattern([a, odd, b])
    assert pat == (3, 1, -1) and keep == [0, 2]
    assert phases == pytest.approx([(2.1, 252.0), (4.9, 795.0), (3.05, 261.0)])


def test_phase_pattern_signs():
    x, cuts = synthetic(1)
    assert phase_pattern(segments_of(x, cuts)) == (5, 1, -1, 1, -1)


@pytest.mark.parametrize("seed", range(4))
def test_boundary_samples_do_not_make_phases(seed):
    """A sensor sample that spans a phase boundary reads a mixture of the two
    levels; the detector gives it a short segment of its own, and folding
    segments under three samples into the closer neighbour leaves one step
    there."""
    rng = np.random.default_rng(50 + seed)
    levels, length = [260.0, 680.0, 740.0, 330.0, 1230.0, 1140.0, 270.0], 8
    x = np.concatenate([np.full(length, v) for v in levels])
    for i in range(1, len(levels)):
        f = rng.uniform(0.2, 0.8)
        x[i * length] = f * levels[i - 1] + (1 - f) * levels[i]
    x += rng.normal(0.0, 5.0, x.size)
    raw = detect_steps(x, noise_std=5.0, min_len=1)
    assert len(raw) > len(levels) - 1
    cuts = merge_short(x, raw, 3)
    assert len(cuts) == len(levels) - 1
    assert all(abs(c - i * length) <= 1 for c, i in zip(cuts, range(1, len(levels))))
    assert phase_pattern(segments_of(x, cuts)) == (7, 1, 1, -1, 1, -1, -1)


def test_merge_short_cases():
    x = np.array([0.0] * 5 + [3.0] + [10.0] * 5 + [9.0, 1.0] + [1.0] * 4)
    assert merge_short(x, [5, 6, 11, 12], 3) == [6, 12]
    assert merge_short(x, [1], 3) == []
    assert merge_short(x, [5, 11], 3) == [5, 11]
    assert merge_short(x, [], 3) == []


def test_noise_from_differences():
    """The estimate ignores the steps: on a long trace with a few large steps
    it lands within 15 % of the noise's sigma, and it is zero without noise."""
    rng = np.random.default_rng(3)
    levels = [260.0, 700.0, 350.0, 1250.0, 1160.0, 270.0]
    x = np.concatenate([np.full(40, v) for v in levels])
    for sigma in (2.0, 5.0, 20.0):
        est = noise_from_differences(x + rng.normal(0.0, sigma, x.size))
        assert abs(est - sigma) <= 0.15 * sigma
    assert noise_from_differences(x) == 0.0
    assert noise_from_differences([1.0]) == 0.0


def test_robust_spread_ignores_an_edge_sample():
    """A noise sample whose last value already belongs to the next phase: the
    standard deviation jumps, the MAD-based spread stays near sigma."""
    rng = np.random.default_rng(5)
    x = 269.0 + rng.normal(0.0, 1.0, 200)
    assert abs(robust_spread(x) - 1.0) <= 0.15
    y = np.append(x[:6], 437.0)
    assert np.std(y) > 50.0 and robust_spread(y) < 3.0
    assert robust_spread([]) == 0.0


def test_sampler_power_from_counter_updates(monkeypatch):
    """The background sampler against a stand-in energy counter that advances
    once every 0.1 s by exactly 300 W x 0.1 s (timestamps in ns, energy in
    units of 15.3 uJ): the mean power between updates and the trace are
    300 W, and an interval with fewer than two updates gives None."""
    import sys
    import threading
    import time
    import types
    from paper_2112_10823_amd.energy import EnergySampler

    res = 15.3e-6  # J per counter unit
    t_start = time.perf_counter()
    lock = threading.Lock()

    def energy_count(_h):
        with lock:
            steps = int((time.perf_counter() - t_start) / 0.1)
        ts = steps * 0.1
        return {"energy_accumulator": int(round(300.0 * ts / res)), "counter_resolution": res * 1e6,
                "timestamp": int(ts * 1e9)}

    fake = types.SimpleNamespace(amdsmi_init=lambda: None,
                                 amdsmi_get_processor_handles=lambda: [0],
                                 amdsmi_get_energy_count=energy_count)
    monkeypatch.setitem(sys.modules, "amdsmi", fake)
    s = EnergySampler(period_s=0.005).start()
    time.sleep(0.75)
    s.stop()
    assert s.ok and len(s.updates) >= 5
    p = s.power_between(s.updates[0][0], s.updates[-1][0])
    assert abs(p - 300.0) <= 300.0 * 1e-3
    t, w = s.trace()
    assert len(w) >= 4 and np.all(np.abs(w - 300.0) <= 300.0 * 1e-3)
    assert s.power_between(s.updates[-1][0] + 1.0, s.updates[-1][0] + 2.0) is None
