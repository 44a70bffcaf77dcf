"""Statistics of energy series: blocking (reblocking) analysis and the
correlated-sampling energy difference.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in float64,
written from the definitions:

* Reblocking (the paper's Sec. II remark that long population-controlled runs
  take their error bars from a reblocking analysis; the analysis is
  Flyvbjerg and Petersen's): level 0 is the series, level k+1 averages
  neighbouring pairs of level k (an odd last element is dropped).  At every
  level with n_k >= 2 values the standard error of the mean is
  sqrt(s_k^2 / n_k) with the unbiased sample variance s_k^2, and its own
  uncertainty is that error / sqrt(2 (n_k - 1)).  The plateau is the first
  level k whose error the next level exceeds by no more than that
  uncertainty; -1 when there is none.
* Correlated sampling (Sec. I, Sec. V: two systems propagated with the same
  auxiliary fields; independent repeats give the error bar): the per-step
  difference d = b - a of each repeat's energy series, its cumulative average
  from step `first` on over the steps where both are finite, and over the
  repeats the mean and the standard error of that cumulative average.
"""
from __future__ import annotations

import numpy as np


def reblock(x, max_levels: int = 64):
    """Returns (mean of the whole series, [standard error per level], plateau
    level or -1)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 1 or x.size < 2 or not np.all(np.isfinite(x)):
        raise ValueError("need a finite 1-d series of at least 2 values")
    mean = float(np.mean(x))
    sems, errs = [], []
    level = x
    while level.size >= 2 and len(sems) < max_levels:
        n = level.size
        var = np.sum((level - np.mean(level)) ** 2) / (n - 1)
        sem = np.sqrt(var / n)
        sems.append(float(sem))
        errs.append(float(sem / np.sqrt(2.0 * (n - 1))))
        m = n // 2
        level = 0.5 * (level[0:2 * m:2] + level[1:2 * m:2])
    plateau = -1
    for k in range(len(sems) - 1):
        if sems[k + 1] - sems[k] <= errs[k]:
            plateau = k
            break
    return mean, sems, plateau


def cs_difference(a, b, first: int = 0):
    """a, b: [repeats][steps] energy series of the two systems (NaN where a
    step has no measurement).  Returns (mean[steps], sem[steps]) of the
    cumulative average of b - a from step `first` on over the repeats (NaN
    before `first`, where no step is finite yet, and sem NaN for 1 repeat)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 2:
        raise ValueError("a and b must be [repeats][steps] of the same shape")
    R, T = a.shape
    cum = np.full((R, T), np.nan)
    for r in range(R):
        s, n = 0.0, 0
        for t in range(T):
            if t >= first and np.isfinite(a[r, t]) and np.isfinite(b[r, t]):
                s += b[r, t] - a[r, t]
                n += 1
            if t >= first and n > 0:
                cum[r, t] = s / n
    mean = np.full(T, np.nan)
    sem = np.full(T, np.nan)
    for t in range(T):
        c = cum[:, t]
        if np.all(np.isfinite(c)):
            mean[t] = np.mean(c)
            if R >= 2:
                sem[t] = np.sqrt(np.sum((c - mean[t]) ** 2) / (R * (R - 1)))
    return mean, sem
