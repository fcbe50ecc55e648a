"""Resampling error bars of ln g over independent runs -- TEST INFRASTRUCTURE ONLY.

The paper determines statistical errors of the stitched DOS by resampling over
independent simulations (end of the parallel-scheme section).  ``jackknife``
is the leave-one-out estimate written from its definition: for R runs and a
bin b, theta_i = mean of ln g_b over the runs other than i, the estimate is
the mean over all runs and its error sqrt((R-1)/R * sum_i (theta_i -
mean_i theta_i)^2).  Bins that some run never visited (-inf) get -inf and NaN.
"""
from __future__ import annotations

import numpy as np


def jackknife(lng_runs):
    x = np.asarray(lng_runs, dtype=np.float64)
    R, B = x.shape
    if R < 2:
        raise ValueError("need at least two runs")
    mean = np.full(B, -np.inf)
    err = np.full(B, np.nan)
    for b in range(B):
        col = x[:, b]
        if not np.all(np.isfinite(col)):
            continue
        theta = np.array([np.mean(np.delete(col, i)) for i in range(R)])
        mean[b] = np.mean(col)
        err[b] = np.sqrt((R - 1) / R * np.sum((theta - np.mean(theta)) ** 2))
    return mean, err
