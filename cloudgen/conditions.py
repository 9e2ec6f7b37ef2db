"""Seeded flow conditions, network inputs and initial network weights for
the learned warm start (inputs only: no solver arithmetic)."""
import numpy as np

from .rng import uniform


def sample_conditions(seed, count, mach=(0.3, 0.6), alpha=(-3.0, 5.0), tau=(0.08, 0.15)):
    """`count` conditions (mach, alpha in degrees, thickness tau), each
    uniform in its range, from three splitmix64 streams of `seed`."""
    m = uniform(seed, count, *mach)
    a = uniform(seed + 1, count, *alpha)
    t = uniform(seed + 2, count, *tau)
    return [dict(mach=float(m[i]), alpha=float(a[i]), tau=float(t[i])) for i in range(count)]


def warm_features(cloud, wall_distance, mach, alpha, tau):
    """Per-point network inputs (x, y, log(wall distance + 1e-3), M, alpha,
    tau), shape (n, 6), caller order."""
    n = cloud.n
    return np.stack([cloud.x, cloud.y, np.log(np.asarray(wall_distance) + 1e-3),
                     np.full(n, mach), np.full(n, alpha), np.full(n, tau)], axis=1)


def glorot_weights(widths, seed):
    """Initial weights in the flat layout (W_l row-major, then b_l): W_l
    uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    parts = []
    for l, (fi, fo) in enumerate(zip(widths[:-1], widths[1:])):
        r = np.sqrt(6.0 / (fi + fo))
        parts.append(uniform(seed + 17 * l, fi * fo, -r, r))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)
