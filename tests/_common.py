"""Shared test inputs: clouds, parameter sets and smooth analytic states."""
import numpy as np

from cloudgen import naca_ocloud

GAMMA = 1.4


def smooth_state(cloud, mach=0.63, alpha_deg=2.0, amp=0.05, gamma=GAMMA):
    """A smooth, positive, non-uniform conserved state (4, n) built from
    primitive fields; the analytic functions are arbitrary test data."""
    x, y = cloud.x, cloud.y
    a = np.radians(alpha_deg)
    rho = 1.0 + amp * np.sin(1.3 * x + 0.4) * np.cos(0.9 * y - 0.2)
    u1 = mach * np.cos(a) * (1.0 + amp * np.cos(0.7 * x - 0.5 * y))
    u2 = mach * np.sin(a) + amp * mach * np.sin(0.8 * x + 1.1 * y)
    p = (1.0 / gamma) * (1.0 + amp * np.cos(0.6 * x + 0.3 * y + 0.1))
    U = np.stack([rho, rho * u1, rho * u2, p / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2)])
    return U


def normwise_rel(a, b):
    """max_p |a_c - b_c| / max_p |b_c| for each row c (rows of zeros: absolute)."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    den = np.abs(b).max(axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b).max(axis=1) / den


_CLOUDS = {}


def cloud(name):
    """Named clouds used across tests (cached)."""
    if name not in _CLOUDS:
        if name == "c1":  # 160 x 60 O-cloud around NACA 0012
            _CLOUDS[name] = naca_ocloud(160, 60)
        elif name == "small":
            _CLOUDS[name] = naca_ocloud(48, 16)
        elif name == "jitter":
            _CLOUDS[name] = naca_ocloud(96, 40, jitter=0.1, seed=2108)
        elif name == "c2":  # 1250 x 2000 = 2.5M points, jittered
            _CLOUDS[name] = naca_ocloud(1250, 2000, jitter=0.1, seed=2108)
        else:
            raise KeyError(name)
    return _CLOUDS[name]
