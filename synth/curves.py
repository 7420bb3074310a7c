"""Seeded point sets on smooth curves in the plane (charge locations of the 2D
potential problem) and seeded real charge vectors."""
import numpy as np


def smooth_curve(n, seed=0, length=4.0, modes=6, amplitude=0.35):
    """n points spread evenly in arc length along a seeded smooth open curve.

    The curve is x(t) = length * t, y(t) = sum_k a_k sin(2 pi k t + phi_k), t in
    [0, 1], with amplitudes a_k = amplitude * u_k / k (u_k uniform in [0.5, 1])
    and random phases: about `length` units wide and under a unit tall, so its
    bounding box is longest along x.  Returns an (n, 2) float64 array ordered
    along the curve."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, modes + 1)
    a = amplitude * rng.uniform(0.5, 1.0, modes) / k
    ph = rng.uniform(0.0, 2.0 * np.pi, modes)
    # fine polyline, then arc-length resampling
    m = max(20 * n, 20000)
    t = np.linspace(0.0, 1.0, m)
    x = length * t
    y = (a[:, None] * np.sin(2.0 * np.pi * k[:, None] * t[None, :] + ph[:, None])).sum(axis=0)
    seg = np.hypot(np.diff(x), np.diff(y))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    # n points at the midpoints of n equal arc-length intervals (no two coincide)
    si = (np.arange(n) + 0.5) * (s[-1] / n)
    return np.stack([np.interp(si, s, x), np.interp(si, s, y)], axis=1)


def real_normal(shape, seed=0):
    """Standard normal float64 array (charges)."""
    return np.random.default_rng(seed).standard_normal(shape)
