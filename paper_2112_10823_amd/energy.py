"""GPU energy measurement and the paper's phase analysis of power traces.

The paper (Section 4) measures board power with current clamps on the 12 V
feeds and an oscilloscope.  The trace is smoothed with an averaging filter,
cut into phases of constant power by a step detector that follows the
variance of the signal and is given a sample of the sensor noise, and the
repeated runs of one experiment that share the most common phase pattern
are averaged; the energy of a phase is its mean power times its duration
(E = P t holds in every table of its Section 5).

Here the sensor is the GPU's own energy accumulator, read through amdsmi.
On MI355X it advances about once per second, so `EnergySampler` polls it in
a background thread and keeps each update with the counter's own
timestamp: the mean power over an interval is the energy between two
updates divided by the time between them, and a power trace is the series
of those ratios.  The analysis functions are plain numpy and do not need a
GPU.
"""
from __future__ import annotations

import threading
import time
from collections import Counter
from dataclasses import dataclass

import numpy as np

__all__ = ["EnergySampler", "moving_average", "robust_spread", "noise_from_differences",
           "detect_steps", "merge_short",
           "Segment", "segments_of",
           "phase_pattern", "most_common_pattern"]


class EnergySampler:
    """Background reader of the amdsmi energy accumulator.

    `updates` holds (host time in s, energy in J, counter time in s) at every
    change of the accumulator.  Unavailable telemetry leaves `ok` False and
    every query returns None."""

    def __init__(self, period_s: float = 0.005, device_index: int = 0):
        self.period = period_s
        self.updates: list[tuple[float, float, float]] = []
        self.ok = False
        self._stop = threading.Event()
        self._th = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            self._h = amdsmi.amdsmi_get_processor_handles()[device_index]
            self._read()
            self.ok = True
        except Exception:
            self._smi = None

    def _read(self):
        e = self._smi.amdsmi_get_energy_count(self._h)
        joules = float(e["energy_accumulator"]) * float(e.get("counter_resolution", 1.0)) * 1e-6
        return joules, float(e.get("timestamp", 0)) * 1e-9

    def _run(self):
        last = None
        while not self._stop.is_set():
            j, ts = self._read()
            if last is None or j != last:
                self.updates.append((time.perf_counter(), j, ts))
                last = j
            time.sleep(self.period)

    def start(self):
        if self.ok and self._th is None:
            self._stop.clear()
            self._th = threading.Thread(target=self._run, daemon=True)
            self._th.start()
        return self

    def stop(self):
        if self._th is not None:
            self._stop.set()
            self._th.join()
            self._th = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    def power_between(self, t0: float, t1: float):
        """Mean power (W) over the counter updates seen inside [t0, t1] (host
        times), or None with fewer than two such updates."""
        u = [x for x in self.updates if t0 <= x[0] <= t1]
        if len(u) < 2 or u[-1][2] <= u[0][2]:
            return None
        return (u[-1][1] - u[0][1]) / (u[-1][2] - u[0][2])

    def trace(self):
        """Power trace from consecutive updates: (host mid-times, W)."""
        u = self.updates
        t = np.array([(a[0] + b[0]) / 2 for a, b in zip(u, u[1:])])
        p = np.array([(b[1] - a[1]) / (b[2] - a[2]) if b[2] > a[2] else np.nan
                      for a, b in zip(u, u[1:])])
        keep = np.isfinite(p)
        return t[keep], p[keep]


def moving_average(x, width: int):
    """Centred averaging filter of odd `width`: y[i] is the mean of the
    samples within width // 2 of i (fewer at the ends)."""
    x = np.asarray(x, dtype=np.float64)
    if width <= 1 or x.size == 0:
        return x.copy()
    h = width // 2
    c = np.concatenate([[0.0], np.cumsum(x)])
    i = np.arange(x.size)
    lo = np.maximum(i - h, 0)
    hi = np.minimum(i + h + 1, x.size)
    return (c[hi] - c[lo]) / (hi - lo)


@dataclass
class Segment:
    start: int   # first sample
    end: int     # one past the last sample
    level: float


def robust_spread(x):
    """Standard deviation of a noise sample estimated from its median
    absolute deviation (1.4826 MAD, exact for Gaussian noise), so that a
    sample taken across the end of the window does not inflate it."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return 0.0
    return float(1.4826 * np.median(np.abs(x - np.median(x))))


def noise_from_differences(x):
    """Standard deviation of the noise on a piecewise-constant signal,
    estimated from its first differences: away from the few steps each
    difference is the difference of two independent noise samples, so the
    median absolute difference, scaled by 1.4826 / sqrt(2), estimates the
    noise's sigma for Gaussian noise and is not moved by the steps."""
    d = np.diff(np.asarray(x, dtype=np.float64))
    if d.size == 0:
        return 0.0
    return float(1.4826 * np.median(np.abs(d)) / np.sqrt(2.0))


def detect_steps(x, noise_std: float, min_len: int = 2, penalty: float | None = None):
    """Change points of a piecewise-constant signal in noise.

    Binary segmentation on the variance: a segment is split where cutting it
    in two removes the most squared deviation from the segment means, if that
    reduction exceeds `penalty` (default 2 ln(n) * 4 noise_std^2, the cost of
    one more step for noise of standard deviation noise_std, which is what
    the noise sample is for); both parts are searched again.  Parts are at
    least `min_len` samples long.  Returns the sorted change indices."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if penalty is None:
        penalty = 8.0 * noise_std ** 2 * np.log(max(n, 2))
    c1 = np.concatenate([[0.0], np.cumsum(x)])
    c2 = np.concatenate([[0.0], np.cumsum(x * x)])

    def sse(a, b):
        m = b - a
        s = c1[b] - c1[a]
        return (c2[b] - c2[a]) - s * s / m

    cuts = []
    todo = [(0, n)]
    while todo:
        a, b = todo.pop()
        if b - a < 2 * min_len:
            continue
        ks = np.arange(a + min_len, b - min_len + 1)
        total = sse(a, b)
        gains = np.array([total - sse(a, k) - sse(k, b) for k in ks])
        best = int(np.argmax(gains))
        if gains[best] > penalty:
            k = int(ks[best])
            cuts.append(k)
            todo.append((a, k))
            todo.append((k, b))
    return sorted(cuts)


def merge_short(x, cuts, min_len: int):
    """Fold every segment shorter than `min_len` samples into the neighbour
    whose level is closer (the shortest first), so that a sample taken across
    a phase boundary, which reads a mixture of the two levels, joins one of
    the two phases instead of standing as a phase of its own.  Returns the
    remaining change indices."""
    x = np.asarray(x, dtype=np.float64)
    cuts = sorted(cuts)
    while cuts:
        bounds = [0] + cuts + [x.size]
        lens = [b - a for a, b in zip(bounds, bounds[1:])]
        k = int(np.argmin(lens))
        if lens[k] >= min_len:
            break
        lv = [float(x[a:b].mean()) for a, b in zip(bounds, bounds[1:])]
        if k == 0:
            drop = 0
        elif k == len(lens) - 1:
            drop = k - 1
        else:
            drop = k - 1 if abs(lv[k] - lv[k - 1]) <= abs(lv[k] - lv[k + 1]) else k
        del cuts[drop]
    return cuts


def segments_of(x, cuts):
    """Segments between the change points with their mean levels."""
    x = np.asarray(x, dtype=np.float64)
    bounds = [0] + list(cuts) + [x.size]
    return [Segment(a, b, float(x[a:b].mean())) for a, b in zip(bounds, bounds[1:]) if b > a]


def phase_pattern(segments):
    """The pattern of a run: its number of phases and the direction of each
    step between consecutive phases."""
    return (len(segments),) + tuple(int(np.sign(b.level - a.level))
                                    for a, b in zip(segments, segments[1:]))


def most_common_pattern(runs):
    """Among runs (each a list of (duration, level) phases with the same
    time base), keep those with the most common pattern and average them
    phase by phase.  Returns (pattern, indices of the kept runs, list of
    (mean duration, mean level) per phase)."""
    pats = [phase_pattern([Segment(0, 0, lv) for _, lv in r]) for r in runs]
    best, _ = Counter(pats).most_common(1)[0]
    keep = [i for i, p in enumerate(pats) if p == best]
    phases = [(float(np.mean([runs[i][k][0] for i in keep])),
               float(np.mean([runs[i][k][1] for i in keep]))) for k in range(best[0])]
    return best, keep, phases
