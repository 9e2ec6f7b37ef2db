"""FP64 reference of the warm start's state map: the network's standardised
primitive fields -> a conserved state the solver can start from.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark may
import this module.  The solver package never does.

The paper starts every run from the freestream; the learned start is an
addition to it, so the map follows the warm-start reading of the design
notes rather than a passage of the paper.  Per point, with the network's
outputs y = (y_rho, y_u1, y_u2, y_p) and the output scaling (mean, std):
    prim  = mean + std * y                      (rho, u1, u2, p)
    a point whose prim has a non-finite component takes the freestream;
    rho  <- max(rho, floor * rho_inf),  p <- max(p, floor * p_inf)
    U     = (rho, rho u1, rho u2, p/(gamma-1) + rho |u|^2 / 2)   (eq. (2))
    a state U with a non-finite component is replaced by the freestream;
    outer points keep the freestream (their far-field condition);
    wall points get the wall condition's projection m <- m - (m.n) n.
The freestream is rho_inf = 1, p_inf = 1/gamma, u_inf = M (cos a, sin a).
"""
import math

import numpy as np

KIND_WALL, KIND_OUTER = 1, 2


def freestream_cons(mach, alpha_deg, gamma=1.4):
    a = alpha_deg * math.pi / 180.0
    u1, u2 = mach * math.cos(a), mach * math.sin(a)
    p = 1.0 / gamma
    return np.array([1.0, u1, u2, p / (gamma - 1.0) + 0.5 * (u1 * u1 + u2 * u2)])


def warm_state(Y, mean, std, floor, kind, nx, ny, mach, alpha_deg, gamma=1.4):
    """Y: (n, 4) network outputs (float32 values, taken exactly into FP64);
    mean, std: 4 float32 values each; floor: fraction of the freestream
    density and pressure below which the state is held; kind, nx, ny: the
    points' kinds and unit normals; mach, alpha_deg: the case's freestream.
    Returns U (4, n)."""
    Y = np.asarray(Y, np.float32).astype(np.float64)
    mean = np.asarray(mean, np.float32).astype(np.float64)
    std = np.asarray(std, np.float32).astype(np.float64)
    n = Y.shape[0]
    Uinf = freestream_cons(mach, alpha_deg, gamma)
    U = np.empty((4, n))
    for p in range(n):
        u = Uinf.copy()
        if kind[p] != KIND_OUTER:
            prim = [mean[c] + std[c] * Y[p, c] for c in range(4)]
            if all(math.isfinite(v) for v in prim):
                rho = max(prim[0], floor * 1.0)
                pr = max(prim[3], floor * (1.0 / gamma))
                v = np.array([rho, rho * prim[1], rho * prim[2],
                              pr / (gamma - 1.0)
                              + 0.5 * rho * (prim[1] * prim[1] + prim[2] * prim[2])])
                if np.all(np.isfinite(v)):
                    u = v
            if kind[p] == KIND_WALL:
                mn = u[1] * nx[p] + u[2] * ny[p]
                u[1] = u[1] - mn * nx[p]
                u[2] = u[2] - mn * ny[p]
        U[:, p] = u
    return U
