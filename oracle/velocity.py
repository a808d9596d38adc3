"""Envelope velocity from a radius time series (TEST INFRASTRUCTURE ONLY).

Sec. 4.2 estimates the front speed from the position of the front at late
times, once the profile has become a travelling wave.  Here the speed is the
ordinary least-squares slope of R(t) over the samples whose radius lies in
the window [r_lo, r_hi] (an early-time cut that skips the transient, and a
late cut that keeps the front away from the no-flux walls).
"""
import numpy as np


def fit_velocity(t, R, r_lo, r_hi, min_points=3):
    """Least-squares slope of R against t over r_lo <= R <= r_hi (FP64).

    Returns (v, npoints); v is nan when fewer than min_points samples qualify.
    """
    t = np.asarray(t, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    sel = (R >= r_lo) & (R <= r_hi)
    k = int(sel.sum())
    if k < min_points:
        return float("nan"), k
    ts, Rs = t[sel], R[sel]
    tm, Rm = ts.mean(), Rs.mean()
    v = float(((ts - tm) * (Rs - Rm)).sum() / ((ts - tm) ** 2).sum())
    return v, k
