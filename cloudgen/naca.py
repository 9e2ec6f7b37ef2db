"""Seeded synthetic point distributions for the q-LSKUM solver.

The paper benchmarks on O-type point distributions around a NACA 0012
airfoil (section 4, 0.625M to 40M points); those files are not public, so
this module builds clouds of the same kind from the analytic NACA 4-digit
thickness law.  It holds geometry and connectivity only: split-stencil
classification, least squares and everything else the method computes live
in the solver and in the oracle, each written separately.

Layout of a cloud (user order): point p = j * ns + i, station i along the
surface (trailing edge, upper surface, leading edge, lower surface, i.e.
counter-clockwise), layer j from the wall (j = 0) to the outer boundary
(j = nr - 1).  The first ns points are therefore the wall points in surface
order.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

from .rng import uniform

KIND_INTERIOR, KIND_WALL, KIND_OUTER = 0, 1, 2


@dataclass
class Cloud:
    x: np.ndarray
    y: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    kind: np.ndarray  # uint8
    nbr_ptr: np.ndarray  # int32 [n+1]
    nbr_idx: np.ndarray  # int32 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.x.shape[0])

    @property
    def nnz(self):
        return int(self.nbr_idx.shape[0])

    def neighbour_counts(self):
        return np.diff(self.nbr_ptr)


def naca_thickness(x, tau):
    """Closed-trailing-edge NACA 4-digit half thickness at chord station x."""
    return 5.0 * tau * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2
                        + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def _upper_half(ns, tau, r_outer):
    """Surface stations, outer-circle stations and normals for i = 0..ns/2."""
    m = ns // 2
    i = np.arange(m + 1)
    phi = 2.0 * np.pi * i / ns
    # stations clustered at the leading edge only: x = 1 - sin(phi/2)
    sx = 1.0 - np.sin(0.5 * phi)
    sx[0], sx[m] = 1.0, 0.0
    sy = naca_thickness(sx, tau)
    sy[0], sy[m] = 0.0, 0.0
    cx = 0.5 + r_outer * np.cos(phi)
    cy = r_outer * np.sin(phi)
    cy[0], cy[m] = 0.0, 0.0
    cx[m] = 0.5 - r_outer
    return sx, sy, cx, cy


def _mirror_full(ns, a_up, sign):
    """Extend an upper-half station array (i = 0..ns/2) to all ns stations by
    the exact mirror x(ns - i) = x(i), y(ns - i) = -y(i)."""
    m = ns // 2
    out = np.empty(ns, dtype=np.float64)
    out[: m + 1] = a_up
    out[m + 1:] = sign * a_up[1:m][::-1]
    return out


def _surface_normals(sx, sy):
    """Outward (into the fluid) unit normal of the counter-clockwise surface
    polygon at each station: (a_y, -a_x) of a = S(i+1) - S(i-1)."""
    ax = np.roll(sx, -1) - np.roll(sx, 1)
    ay = np.roll(sy, -1) - np.roll(sy, 1)
    norm = np.hypot(ax, ay)
    return ay / norm, -ax / norm


def naca_ocloud(ns, nr, tau=0.12, r_outer=15.0, q_stretch=1.08 ** 59,
                jitter=0.0, seed=2108, stencil="box", box_halfwidth=2,
                radius_factor=2.5, max_neighbours=25, smooth=1.0 / 40.0, progress=None):
    """O-type cloud of ns x nr points around a NACA 00xx airfoil.

    Layer j sits at the blend parameter w_j = (Q^{t_j} - 1)/(Q - 1),
    t_j = j/(nr-1), so that the first layers grow geometrically by
    Q^{1/(nr-1)} per layer (1.08 at nr = 60).  Each column i is the cubic
    Hermite curve from the surface station S_i to the far-field station C_i
    (circle of radius r_outer about mid-chord) that meets the circle radially
    and leaves the wall along the wall normal, smoothed over a window of
    `smooth * ns` stations so that columns fan out gradually from the sharp
    trailing edge; away from the trailing edge the lattice is close to
    orthogonal next to the wall.  The
    lower half is an exact mirror of the upper half, so a symmetric
    airfoil's cloud is mirror-exact bit for bit when no jitter is applied.

    Frames: each point's unit normal is perpendicular to its own layer
    (outward), so at the wall it is the wall normal and everywhere it is
    aligned with the local lattice.

    Connectivity: `stencil="box"` takes every lattice point within 2.5 local
    spacings along each lattice direction, i.e. the (2k+1) x (2k+1) lattice
    box with k = box_halfwidth (24 neighbours in the interior, one-sided at
    the wall and the outer boundary; never above `max_neighbours`).
    Where a split half plane the residual needs is degenerate (fewer than two
    points or nearly collinear, as next to the sharp trailing edge), the
    nearest points of that half plane are added.
    `stencil="radius"` instead takes every point closer than radius_factor
    times the largest lattice edge at the point, capped at max_neighbours.

    `jitter` moves interior points by U(-jitter, jitter) times the local
    tangential and radial lattice spacing (splitmix64 stream seeded with
    `seed`: two draws per interior point in user order, tangential first).

    `progress`, if given, is called with a short message after each chunk
    of work (large clouds take minutes).
    """
    if ns % 2 or ns < 8 or nr < 3:
        raise ValueError("ns must be even and >= 8, nr >= 3")
    m = ns // 2
    sx_u, sy_u, cx_u, cy_u = _upper_half(ns, tau, r_outer)
    sx = _mirror_full(ns, sx_u, 1.0)
    sy = _mirror_full(ns, sy_u, -1.0)
    cx = _mirror_full(ns, cx_u, 1.0)
    cy = _mirror_full(ns, cy_u, -1.0)
    wnx_u, wny_u = _surface_normals(sx, sy)
    wnx = _mirror_full(ns, wnx_u[: m + 1], 1.0)
    wny = _mirror_full(ns, wny_u[: m + 1], -1.0)
    wny[0], wny[m] = 0.0, 0.0
    # outward radial direction of the far-field circle
    rx = _mirror_full(ns, (cx_u - 0.5) / r_outer, 1.0)
    ry = _mirror_full(ns, cy_u / r_outer, -1.0)

    t = np.arange(nr, dtype=np.float64) / (nr - 1)
    w = (q_stretch ** t - 1.0) / (q_stretch - 1.0)
    w[0], w[-1] = 0.0, 1.0
    h0 = (2 * w ** 3 - 3 * w ** 2 + 1)[:, None]
    h1 = (3 * w ** 2 - 2 * w ** 3)[:, None]
    h2 = (w ** 3 - 2 * w ** 2 + w)[:, None]
    h3 = (w ** 3 - w ** 2)[:, None]
    span = np.hypot(cx - sx, cy - sy)[None, :]
    dnx, dny = _departure_directions(wnx, wny, smooth)
    X = h0 * sx[None, :] + h1 * cx[None, :] + h2 * span * dnx[None, :] + h3 * span * rx[None, :]
    Y = h0 * sy[None, :] + h1 * cy[None, :] + h2 * span * dny[None, :] + h3 * span * ry[None, :]
    X[0], Y[0] = sx, sy
    X[-1], Y[-1] = cx, cy
    # restore the exact mirror of the lower half row by row
    X[:, m + 1:] = X[:, 1:m][:, ::-1]
    Y[:, m + 1:] = -Y[:, 1:m][:, ::-1]
    Y[:, 0] = 0.0
    Y[:, m] = 0.0

    # local lattice spacings on the unjittered lattice
    et_next = np.hypot(np.roll(X, -1, axis=1) - X, np.roll(Y, -1, axis=1) - Y)
    et_prev = np.roll(et_next, 1, axis=1)
    er_next = np.full_like(X, 0.0)
    er_next[:-1] = np.hypot(X[1:] - X[:-1], Y[1:] - Y[:-1])
    er_prev = np.full_like(X, 0.0)
    er_prev[1:] = er_next[:-1]

    # layer-aligned frames: outward normal of each layer polygon
    ax = np.roll(X, -1, axis=1) - np.roll(X, 1, axis=1)
    ay = np.roll(Y, -1, axis=1) - np.roll(Y, 1, axis=1)
    an = np.hypot(ax, ay)
    NX, NY = ay / an, -ax / an
    NX[:, m + 1:] = NX[:, 1:m][:, ::-1]
    NY[:, m + 1:] = -NY[:, 1:m][:, ::-1]
    NY[:, 0] = 0.0
    NY[:, m] = 0.0
    NX[:, 0], NX[:, m] = 1.0, -1.0

    kind = np.zeros((nr, ns), dtype=np.uint8)
    kind[0, :] = KIND_WALL
    kind[-1, :] = KIND_OUTER

    xs, ys = X.copy(), Y.copy()
    if jitter > 0.0:
        h_t = 0.5 * (et_next + et_prev)
        h_r = 0.5 * (er_next + er_prev)
        n_int = (nr - 2) * ns
        r = uniform(seed, 2 * n_int, -jitter, jitter).reshape(nr - 2, ns, 2)
        tx, ty = NY[1:-1], -NX[1:-1]
        dt_ = r[..., 0] * h_t[1:-1]
        dr_ = r[..., 1] * h_r[1:-1]
        xs[1:-1] = X[1:-1] + dt_ * tx + dr_ * NX[1:-1]
        ys[1:-1] = Y[1:-1] + dt_ * ty + dr_ * NY[1:-1]

    x = xs.reshape(-1)
    y = ys.reshape(-1)
    ii = np.tile(np.arange(ns), nr)
    jj = np.repeat(np.arange(nr), ns)
    key = _mirror_tie_key(ii, jj, ns, y)
    NXf, NYf = NX.reshape(-1).copy(), NY.reshape(-1).copy()
    kindf = kind.reshape(-1)
    if stencil == "box":
        ptr, idx = lattice_box_neighbours(x, y, ns, nr, box_halfwidth, max_neighbours,
                                          progress=progress)
        ptr, idx = enrich_half_planes(x, y, NXf, NYf, kindf, ptr, idx, max_neighbours,
                                      progress=progress)
    elif stencil == "radius":
        h_p = np.maximum.reduce([et_next, et_prev, er_next, er_prev])
        ptr, idx = radius_neighbours(x, y, radius_factor * h_p.reshape(-1), max_neighbours,
                                     tie_key=key)
    else:
        raise ValueError(stencil)
    cloud = Cloud(x=x, y=y, nx=NXf, ny=NYf, kind=kindf, nbr_ptr=ptr, nbr_idx=idx,
                  meta=dict(ns=ns, nr=nr, tau=tau, r_outer=r_outer, jitter=jitter,
                            seed=seed, stencil=stencil, kind="naca_ocloud"))
    return cloud




def naca_ocloud_cached(path, ns, nr, **kw):
    """naca_ocloud(ns, nr, **kw), kept in an uncompressed .npz at `path`:
    loaded from there when the file holds a cloud made with the same
    arguments, else built and written (large clouds take minutes to build
    and seconds to load).  `progress` is passed through and not stored."""
    import json
    import os
    progress = kw.pop("progress", None)
    key = json.dumps(dict(ns=ns, nr=nr, **kw), sort_keys=True)
    if path and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            if str(z["key"]) == key:
                c = Cloud(x=z["x"], y=z["y"], nx=z["nx"], ny=z["ny"], kind=z["kind"],
                          nbr_ptr=z["nbr_ptr"], nbr_idx=z["nbr_idx"],
                          meta=json.loads(str(z["meta"])))
                if progress is not None:
                    progress(f"cloud loaded from {path}")
                return c
    c = naca_ocloud(ns, nr, progress=progress, **kw)
    if path:
        tmp = path + ".tmp.npz"
        np.savez(tmp, key=np.array(key), meta=np.array(json.dumps(c.meta, sort_keys=True)),
                 x=c.x, y=c.y, nx=c.nx, ny=c.ny, kind=c.kind, nbr_ptr=c.nbr_ptr,
                 nbr_idx=c.nbr_idx)
        os.replace(tmp, path)
        if progress is not None:
            progress(f"cloud written to {path}")
    return c

def _departure_directions(wnx, wny, smooth):
    """Wall normals with their angle smoothed (periodic Gaussian of width
    smooth * ns stations) about the uniform angle 2 pi i / ns."""
    ns = wnx.shape[0]
    th = np.unwrap(np.arctan2(wny, wnx))
    base = 2.0 * np.pi * np.arange(ns) / ns
    dev = th - base
    dev -= 2.0 * np.pi * np.round(dev[0] / (2.0 * np.pi))
    sig = max(smooth * ns, 1e-9)
    k = np.arange(-ns // 2, ns // 2)
    ker = np.exp(-0.5 * (k / sig) ** 2)
    ker /= ker.sum()
    sm = np.real(np.fft.ifft(np.fft.fft(dev) * np.fft.fft(np.fft.ifftshift(ker))))
    m = ns // 2
    sm[m + 1:] = -sm[1:m][::-1]
    sm[0] = 0.0
    sm[m] = 0.0
    th2 = base + sm
    return np.cos(th2), np.sin(th2)


def _half_plane_quality(x, y, nx, ny, kind, ptr, idx, chunk=1 << 20, progress=None):
    """Per point and half plane (s<0, s>0, n<0, n>0 in the point's frame),
    the count and the normalised determinant det/(sum ds^2 + sum dn^2)^2 of
    the 2x2 moment matrix of the neighbour offsets in that half plane, and
    whether the half plane is needed (interior: all four; wall: all but
    n<0, which lies in the body; outer: none).  Points are processed in
    chunks so that the per-entry temporaries stay small."""
    n = x.shape[0]
    cnt = np.zeros((4, n))
    qual = np.zeros((4, n))
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        m_ = hi - lo
        loc = np.repeat(np.arange(m_), np.diff(ptr[lo:hi + 1]))
        owner = loc + lo
        nb = idx[int(ptr[lo]):int(ptr[hi])]
        dx = x[nb] - x[owner]
        dy = y[nb] - y[owner]
        ds = dx * ny[owner] - dy * nx[owner]
        dn = dx * nx[owner] + dy * ny[owner]
        tie = 1e-24 * (dx * dx + dy * dy)
        halves = [(ds * ds > tie) & (ds < 0), (ds * ds > tie) & (ds > 0),
                  (dn * dn > tie) & (dn < 0), (dn * dn > tie) & (dn > 0)]
        for h, m in enumerate(halves):
            w = m.astype(np.float64)
            ss = np.bincount(loc, w * ds * ds, minlength=m_)
            sn = np.bincount(loc, w * ds * dn, minlength=m_)
            nn = np.bincount(loc, w * dn * dn, minlength=m_)
            cnt[h, lo:hi] = np.bincount(loc, w, minlength=m_)
            sc = ss + nn
            qual[h, lo:hi] = np.where(sc > 0, (ss * nn - sn * sn) / np.where(sc > 0, sc * sc, 1.0),
                                      0.0)
        if progress is not None:
            progress(f"split half planes {hi}/{n}")
    need = np.ones((4, n), dtype=bool)
    need[:, kind == KIND_OUTER] = False
    need[2, kind == KIND_WALL] = False
    return cnt, qual, need


def enrich_half_planes(x, y, nx, ny, kind, ptr, idx, cap, min_quality=1e-4, min_count=3,
                       pool=1024, progress=None):
    """Add neighbours where a needed split half plane is poorly conditioned
    (fewer than `min_count` points or a normalised determinant below
    `min_quality`, e.g. the on-axis points behind a sharp trailing edge): the
    nearest points of that half plane not yet in the stencil that improve
    it, one at a time, until both bounds hold (at most `cap` neighbours)."""
    cnt, qual, need = _half_plane_quality(x, y, nx, ny, kind, ptr, idx, progress=progress)
    bad = np.flatnonzero(np.any(need & ((cnt < min_count) | (qual <= min_quality)), axis=0))
    if progress is not None:
        progress(f"split half planes checked: {bad.size} points to repair")
    if bad.size == 0:
        return ptr, idx
    tree = cKDTree(np.stack([x, y], axis=1))
    _, cand = tree.query(np.stack([x[bad], y[bad]], axis=1), k=min(pool, x.shape[0]))
    lists = {int(p): list(idx[ptr[p]:ptr[p + 1]]) for p in bad}

    def local(p, i):
        ex, ey = x[i] - x[p], y[i] - y[p]
        return ex * ny[p] - ey * nx[p], ex * nx[p] + ey * ny[p]

    def quality(vs):
        if len(vs) < 2:
            return -1.0
        a = np.array(vs)
        ss, sn, nn = (a[:, 0] ** 2).sum(), (a[:, 0] * a[:, 1]).sum(), (a[:, 1] ** 2).sum()
        return (ss * nn - sn * sn) / (ss + nn) ** 2

    for row, p in enumerate(bad):
        p = int(p)
        cur = lists[p]
        for h in range(4):
            if not need[h, p]:
                continue
            sel = [v for v in (local(p, i) for i in cur) if _in_half(v, h)]
            qcur = quality(sel)
            while qcur <= min_quality or len(sel) < min_count:
                # the nearest few candidates of this half plane; take the one
                # that conditions it best
                opts = []
                for c_ in cand[row]:
                    c_ = int(c_)
                    if c_ == p or c_ in cur:
                        continue
                    v = local(p, c_)
                    if _in_half(v, h):
                        opts.append((c_, v))
                        if len(opts) == 8:
                            break
                if not opts or len(cur) >= cap:
                    raise ValueError(f"cannot repair split stencil {h} of point {p}")
                best = max(opts, key=lambda o: quality(sel + [o[1]]))
                cur.append(best[0])
                sel.append(best[1])
                qcur = quality(sel)
    counts = np.diff(ptr).astype(np.int64)
    for p in bad:
        counts[p] = len(lists[int(p)])
    nptr = np.zeros(x.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=nptr[1:])
    nidx = np.empty(nptr[-1], dtype=np.int32)
    # untouched rows between repaired ones are copied as blocks (bad is sorted)
    nxt = 0
    for p in bad:
        p = int(p)
        nidx[nptr[nxt]:nptr[p]] = idx[ptr[nxt]:ptr[p]]
        nidx[nptr[p]:nptr[p + 1]] = lists[p]
        nxt = p + 1
    nidx[nptr[nxt]:] = idx[ptr[nxt]:]
    return nptr.astype(np.int32), nidx


def _in_half(v, h):
    ds, dn = v
    tie = 1e-24 * (ds * ds + dn * dn)
    if h == 0:
        return ds * ds > tie and ds < 0
    if h == 1:
        return ds * ds > tie and ds > 0
    if h == 2:
        return dn * dn > tie and dn < 0
    return dn * dn > tie and dn > 0

def lattice_box_neighbours(x, y, ns, nr, k, cap, tie_key=None, chunk=1 << 20, progress=None):
    """Neighbours of lattice point (i, j): every (i+a mod ns, j+b) with
    |a|, |b| <= k, b inside the layer range, sorted by distance, ties by layer
    offset b and then by the station offset a signed by the side of the
    x axis the point lies on (so mirror images list mirrored neighbours in
    the same order); at most `cap` (those strictly closer than the first one
    dropped).  Points are processed in chunks of `chunk`."""
    n = ns * nr
    offs = np.array([(a, b) for b in range(-k, k + 1) for a in range(-k, k + 1) if (a, b) != (0, 0)])
    m = offs.shape[0]
    # per side, offsets pre-ordered by the tie key (b, side * a)
    order_up = np.lexsort((offs[:, 0], offs[:, 1]))
    order_lo = np.lexsort((-offs[:, 0], offs[:, 1]))
    a_up, b_up = offs[order_up, 0][None, :], offs[order_up, 1][None, :]
    a_lo, b_lo = offs[order_lo, 0][None, :], offs[order_lo, 1][None, :]
    counts = np.empty(n, dtype=np.int64)
    parts = []
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        p = np.arange(lo, hi)
        ip, jp = p % ns, p // ns
        up = (np.where(y[lo:hi] < 0.0, -1, 1) > 0)[:, None]
        A = np.where(up, a_up, a_lo)
        B = np.where(up, b_up, b_lo)
        jn = jp[:, None] + B
        valid = (jn >= 0) & (jn < nr)
        cols = np.where(valid, jn, 0) * ns + (ip[:, None] + A) % ns
        dx = x[cols] - x[lo:hi, None]
        dy = y[cols] - y[lo:hi, None]
        d2 = np.where(valid, dx * dx + dy * dy, np.inf)
        o = np.argsort(d2, axis=1, kind="stable")
        d2 = np.take_along_axis(d2, o, axis=1)
        cols = np.take_along_axis(cols, o, axis=1)
        keep = np.isfinite(d2)
        if m > cap:
            cut = d2[:, cap][:, None]
            keep &= ~np.isfinite(cut) | (d2 < cut)
        counts[lo:hi] = keep.sum(axis=1)
        parts.append(cols[keep].astype(np.int32))
        if progress is not None:
            progress(f"lattice neighbours {hi}/{n}")
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr.astype(np.int32), np.concatenate(parts)


def _mirror_tie_key(ii, jj, ns, y):
    """Tie-break key for neighbours at equal distance: layer offset first, then
    the station offset signed so that a point and its mirror image order their
    mirrored neighbours alike."""
    def key(p, nb):
        dj = jj[nb] - jj[p]
        di = (ii[nb] - ii[p] + ns // 2) % ns - ns // 2
        side = np.where(y[p] < 0.0, -1, 1)
        return dj, side * di
    return key


def radius_neighbours(x, y, radius, cap, tie_key=None, chunk=1 << 20):
    """CSR neighbour lists: every other point closer than radius[p], keeping
    only those strictly closer than the (cap+1)-th nearest when more than
    `cap` qualify.  Each list is sorted by distance, ties by `tie_key`."""
    n = x.shape[0]
    pts = np.stack([x, y], axis=1)
    tree = cKDTree(pts)
    k = min(cap + 2, n)
    counts = np.zeros(n, dtype=np.int64)
    parts = []
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        d, nb = tree.query(pts[lo:hi], k=k, workers=-1)
        p = np.arange(lo, hi)[:, None]
        notself = nb != p
        # distances squared recomputed exactly from coordinates
        dx = x[nb] - x[p]
        dy = y[nb] - y[p]
        d2 = dx * dx + dy * dy
        d2 = np.where(notself, d2, np.inf)
        order = np.argsort(d2, axis=1, kind="stable")
        d2 = np.take_along_axis(d2, order, axis=1)
        nb = np.take_along_axis(nb, order, axis=1)
        r2 = (radius[lo:hi] ** 2)[:, None]
        keep = d2 < r2
        if d2.shape[1] > cap:
            d_cut = d2[:, cap][:, None]  # (cap+1)-th nearest other point
            over = np.isfinite(d_cut) & (d_cut < r2)
            keep &= ~over | (d2 < d_cut)
        keep &= np.isfinite(d2)
        rows = np.repeat(np.arange(lo, hi), keep.sum(axis=1))
        cols = nb[keep]
        dd = d2[keep]
        if tie_key is not None:
            k1, k2 = tie_key(rows, cols)
            o = np.lexsort((k2, k1, dd, rows))
        else:
            o = np.lexsort((cols, dd, rows))
        rows, cols = rows[o], cols[o]
        counts[lo:hi] = np.bincount(rows - lo, minlength=hi - lo)
        parts.append(cols.astype(np.int32))
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    if ptr[-1] >= 2 ** 31:
        raise ValueError("neighbour count exceeds int32 indexing")
    return ptr.astype(np.int32), np.concatenate(parts) if parts else np.zeros(0, np.int32)


def five_point_cloud(h=0.05):
    """Five points, complete connectivity, all interior, global frame
    (n = (0, 1)): P0 at the origin and four neighbours placed so that each
    of P0's split stencils holds exactly two non-collinear points."""
    x = np.array([0.0, h, -h / 2, -h, h / 2])
    y = np.array([0.0, h / 2, h, -h / 2, -h])
    ptr = np.arange(0, 21, 4, dtype=np.int32)
    idx = np.array([j for i in range(5) for j in range(5) if j != i], dtype=np.int32)
    return Cloud(x=x, y=y, nx=np.zeros(5), ny=np.ones(5), kind=np.zeros(5, np.uint8),
                 nbr_ptr=ptr, nbr_idx=idx, meta=dict(kind="five_point", h=h))


def random_cloud(n, seed, k=12, wall_fraction=0.1, margin=0.15):
    """Poisson cloud in the unit square with k-nearest connectivity (repaired
    where a needed split half plane is degenerate) and random unit frames.
    Points within `margin` of the square's edge are outer points; a random
    fraction of the rest are wall points."""
    u = uniform(seed, 5 * n, 0.0, 1.0).reshape(n, 5)
    x, y = u[:, 0].copy(), u[:, 1].copy()
    th = 2.0 * np.pi * u[:, 2]
    nx, ny = np.cos(th), np.sin(th)
    kind = np.where(u[:, 3] < wall_fraction, KIND_WALL, KIND_INTERIOR).astype(np.uint8)
    edge = (x < margin) | (x > 1 - margin) | (y < margin) | (y > 1 - margin)
    kind[edge] = KIND_OUTER
    ptr, idx = radius_neighbours(x, y, np.full(n, np.inf), k)
    ptr, idx = enrich_half_planes(x, y, nx, ny, kind, ptr, idx, k + 12)
    return Cloud(x=x, y=y, nx=nx, ny=ny, kind=kind, nbr_ptr=ptr, nbr_idx=idx,
                 meta=dict(kind="random", seed=seed, k=k))


def rotate_cloud(cloud, theta):
    """Rigidly rotate positions and frames by theta (radians)."""
    c, s = np.cos(theta), np.sin(theta)
    return Cloud(x=c * cloud.x - s * cloud.y, y=s * cloud.x + c * cloud.y,
                 nx=c * cloud.nx - s * cloud.ny, ny=s * cloud.nx + c * cloud.ny,
                 kind=cloud.kind.copy(), nbr_ptr=cloud.nbr_ptr.copy(),
                 nbr_idx=cloud.nbr_idx.copy(), meta=dict(cloud.meta, rotated=theta))


def surface_arclength_check(cloud):
    """Perimeter of the wall polygon (wall points in user order)."""
    w = np.flatnonzero(cloud.kind == KIND_WALL)
    xw, yw = cloud.x[w], cloud.y[w]
    return float(np.sum(np.hypot(np.roll(xw, -1) - xw, np.roll(yw, -1) - yw)))
