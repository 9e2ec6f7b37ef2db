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


def mixed_g_bound(c, q, g):
    """Per-row bound (8 rows: q_x then q_y components) on normwise_rel of the
    mixed path's q-derivatives against FP64 ones.  Their data are q and the
    iterates rounded to FP32 (relative error <= 2^-24), so each difference
    q_i - q_p is off by at most 2^-23 max|q| and a least-squares derivative
    over offsets no shorter than the smallest neighbour distance d_min by
    about 2^-23 max|q| / d_min; the factor 8 covers the stencils' geometry
    and the inner iterations (which contract).  q: (4, n), g: (8, n)."""
    owner = np.repeat(np.arange(c.n), np.diff(c.nbr_ptr))
    dmin = np.hypot(c.x[c.nbr_idx] - c.x[owner], c.y[c.nbr_idx] - c.y[owner]).min()
    qmax = np.abs(q).max(axis=1)
    return 8.0 * 2.0 ** -23 * np.concatenate([qmax, qmax]) / dmin / np.abs(g).max(axis=1)


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


def dependency_subcloud(c, centres, depth):
    """The points reachable from `centres` in at most `depth` hops along each
    point's own neighbour list, as a cloud of their own.

    Points fewer than `depth` hops out keep their full lists in the stored
    order.  The outermost ring is made of outer (held) points; what they
    compute never reaches a centre, so their lists only have to be valid
    stencils: every other member within two hops, in index order (the
    members among their own neighbours alone can be one-sided or collinear).
    Every value the method computes at a centre that depends on the state
    only within depth - 1 hops (q-derivatives after k inner iterations reach
    k + 1 hops, the flux residual k + 2) is then the same computation on the
    sub-cloud as on the whole cloud.  Returns the sub-cloud, the member
    indices (ascending, the sub-cloud's point order) and the sub-cloud index
    of each centre."""
    from cloudgen import Cloud, KIND_OUTER
    ptr, idx = c.nbr_ptr, c.nbr_idx
    hop = np.full(c.n, -1, dtype=np.int8)
    front = np.unique(np.asarray(centres, dtype=np.int64))
    hop[front] = 0
    for r in range(1, depth + 1):
        nb = np.unique(np.concatenate([idx[ptr[p]:ptr[p + 1]] for p in front]))
        nb = nb[hop[nb] < 0]
        hop[nb] = r
        front = nb
    members = np.flatnonzero(hop >= 0)
    lists, kind = [], c.kind[members].copy()
    for k, p in enumerate(members):
        nb = idx[ptr[p]:ptr[p + 1]]
        if hop[p] == depth:
            two = np.concatenate([nb] + [idx[ptr[i]:ptr[i + 1]] for i in nb])
            two = np.unique(two[hop[two] >= 0])
            nb = two[two != p]
            kind[k] = KIND_OUTER
        lists.append(np.searchsorted(members, nb))
    sptr = np.zeros(members.size + 1, dtype=np.int32)
    np.cumsum([len(v) for v in lists], out=sptr[1:])
    sub = Cloud(x=c.x[members], y=c.y[members], nx=c.nx[members], ny=c.ny[members], kind=kind,
                nbr_ptr=sptr, nbr_idx=np.concatenate(lists).astype(np.int32))
    return sub, members, np.searchsorted(members, np.asarray(centres, dtype=np.int64))


def sample_points(c, count, seed):
    """Seeded sample of points for checks at full size: `count` uniformly
    drawn points plus the wall and next-to-outer points at the trailing and
    leading edges and the points with the longest neighbour lists."""
    from cloudgen import uniform01
    n = c.n
    pick = np.minimum((uniform01(seed, count) * n).astype(np.int64), n - 1)
    special = []
    ns = c.meta.get("ns")
    nr = c.meta.get("nr")
    if ns and nr:
        for i in (0, 1, ns // 2, ns - 1):
            for j in (0, 1, nr // 2, nr - 2):
                special.append(j * ns + i)
    deg = np.diff(c.nbr_ptr)
    special.extend(np.argsort(deg, kind="stable")[-8:].tolist())
    return np.unique(np.concatenate([pick, np.array(special, dtype=np.int64)]))
