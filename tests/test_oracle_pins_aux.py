"""Pins of the oracle's time step, residual norm, forces and limiter against
what the mathematics fixes independently of the oracle's own formulas.

  timestep()   : a binary-exact hand case (every operation exact in IEEE
                 double), and exact scaling laws: dt is linear in the CFL
                 number and in a uniform stretch of the cloud, and inversely
                 proportional to the signal speed |u| + c (Algorithm 1; the
                 local-time-step reading)
  residue()    : closed-form root mean square over the updated (interior and
                 wall) points of a hand-built residual (Algorithm 1; the
                 residual-norm reading)
  forces       : a uniform pressure exerts no force on a closed regular
                 polygon; a linear pressure field p = p_inf + a y (or b x)
                 exerts F = -(0, a A) (or -(b A, 0)) on a body of area A
                 (divergence theorem), reached at second order in the surface
                 spacing on a non-uniformly sampled ellipse; lift and drag
                 rotate with the incidence (the postprocessor reading)
  limiter      : properties of the Venkatakrishnan limiter (J. Comput. Phys.
                 118, 1995) that do not depend on how it is written: without
                 eps the limited increment stays inside the point's bounds,
                 phi follows min(1, D/delta) at small D/delta (slope 1),
                 phi -> 1 as the bounds (or eps) grow, phi = 1 at a zero
                 increment, mirror symmetry, eps^2 homogeneous of degree 3
                 in K and in |P_i - P_0|; on a cloud, eq. (28) gives for a
                 linear field its values half an edge either side of P_0
                 (at P_0 + d/2 and P_0 - d/2, d = P_i - P_0)
"""
import math

import numpy as np
import pytest

import oracle
from cloudgen import Cloud, KIND_INTERIOR, KIND_OUTER, KIND_WALL, naca_ocloud
from tests._common import smooth_state


def _complete_cloud(x, y, kind=None, nx=None, ny=None):
    """Every point a neighbour of every other, in index order."""
    n = len(x)
    idx = np.concatenate([[j for j in range(n) if j != p] for p in range(n)]).astype(np.int32)
    ptr = (np.arange(n + 1) * (n - 1)).astype(np.int32)
    kind = np.zeros(n, np.uint8) if kind is None else np.asarray(kind, np.uint8)
    nx = np.zeros(n) if nx is None else np.asarray(nx, np.float64)
    ny = np.ones(n) if ny is None else np.asarray(ny, np.float64)
    return Cloud(x=np.asarray(x, np.float64), y=np.asarray(y, np.float64), nx=nx, ny=ny,
                 kind=kind, nbr_ptr=ptr, nbr_idx=idx)


def _cons(rho, u1, u2, p, gamma):
    return np.array([rho, rho * u1, rho * u2, p / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2)])


# ------------------------------------------------------------- timestep
def test_timestep_binary_exact_hand_case(oracle_lib):
    """gamma = 5/4, rho = 5/4, u = (3/4, 1), p = 1: |u| = 5/4 and c = 1 exactly;
    CFL = 1/2.  Point 0 sees neighbours at 9/8, 5/4 and 2 (nearest 9/8):
    dt = (1/2)(9/8)/(9/4) = 1/4.  Point 3 is at rest (|u| + c = 1) with its
    nearest neighbour at 2: dt = 1.  Every operation is exact in binary, so
    the values are bit-exact; the largest distance, the sound speed without
    gamma, or a missing CFL would each give another value."""
    g = 1.25
    c = _complete_cloud([0.0, 1.125, 0.75, -2.0], [0.0, 0.0, 1.0, 0.0])
    o = oracle.Oracle(c, oracle.params(gamma=g, cfl=0.5))
    U = np.stack([_cons(1.25, 0.75, 1.0, 1.0, g)] * 3 + [_cons(1.25, 0.0, 0.0, 1.0, g)], axis=1)
    assert U[3, 0] == 4.9765625  # p/(gamma-1) + rho|u|^2/2 = 4 + 0.9765625, exact
    dt = o.timestep(U)
    assert dt[0] == 0.25
    assert dt[3] == 1.0
    # points 1 and 2: nearest neighbour distance over the same signal speed
    d1 = min(1.125, math.hypot(0.375, 1.0), 3.125)
    assert dt[1] == pytest.approx(0.5 * d1 / 2.25, rel=1e-15)
    d2 = min(1.25, math.hypot(0.375, 1.0), math.hypot(2.75, 1.0))
    assert dt[2] == pytest.approx(0.5 * d2 / 2.25, rel=1e-15)


def test_timestep_scaling_laws(oracle_lib):
    """Scaling by powers of two is exact in binary, so each law holds bit for
    bit: dt(2 CFL) = 2 dt; dt on the cloud stretched by 2 = 2 dt; doubling
    every velocity and the sound speed (momentum x2, energy x4) halves dt."""
    c = naca_ocloud(48, 16)
    U = smooth_state(c)
    o = oracle.Oracle(c, oracle.params(cfl=0.2))
    dt = o.timestep(U)
    assert np.all(dt > 0) and np.all(np.isfinite(dt))
    o.set_params(cfl=0.4)
    assert np.array_equal(o.timestep(U), 2.0 * dt)
    big = Cloud(x=2.0 * c.x, y=2.0 * c.y, nx=c.nx, ny=c.ny, kind=c.kind, nbr_ptr=c.nbr_ptr,
                nbr_idx=c.nbr_idx)
    ob = oracle.Oracle(big, oracle.params(cfl=0.2))
    assert np.array_equal(ob.timestep(U), 2.0 * dt)
    fast = U * np.array([1.0, 2.0, 2.0, 4.0])[:, None]
    o.set_params(cfl=0.2)
    assert np.array_equal(o.timestep(fast), 0.5 * dt)


# -------------------------------------------------------------- residue
def test_residue_closed_form(oracle_lib):
    """kinds (interior, wall, outer, interior, outer, wall): the norm is over
    the four updated points only, sqrt((1 + 1 + 9 + 25)/4) = 3 for the first
    row; the outer points' entries (100, -50) must not enter, nor count."""
    kind = [KIND_INTERIOR, KIND_WALL, KIND_OUTER, KIND_INTERIOR, KIND_OUTER, KIND_WALL]
    c = _complete_cloud(np.arange(6.0), np.arange(6.0) ** 2, kind=kind)
    o = oracle.Oracle(c)
    R = np.array([[1.0, 1.0, 100.0, 3.0, -50.0, 5.0],
                  [2.0, 2.0, 100.0, 6.0, -50.0, 10.0],
                  [0.0, 0.0, 100.0, 0.0, -50.0, 4.0],
                  [-1.0, -1.0, 100.0, -3.0, -50.0, -5.0]])
    assert np.array_equal(o.residue(R), [3.0, 6.0, 2.0, 3.0])


def test_residue_uniform_value(oracle_lib):
    """A residual equal to v at every updated point has norm |v| whatever
    the outer points hold."""
    c = naca_ocloud(48, 16)
    o = oracle.Oracle(c)
    R = np.where(c.kind == KIND_OUTER, 7.0, -0.375)[None, :].repeat(4, axis=0)
    assert np.array_equal(o.residue(R), [0.375] * 4)


# --------------------------------------------------------------- forces
def _ring(xs, ys, nxs, nys):
    n = len(xs)
    ptr = (np.arange(n + 1) * 2).astype(np.int32)
    idx = np.array([[(p - 1) % n, (p + 1) % n] for p in range(n)], np.int32).ravel()
    return Cloud(x=np.asarray(xs), y=np.asarray(ys), nx=np.asarray(nxs), ny=np.asarray(nys),
                 kind=np.full(n, KIND_WALL, np.uint8), nbr_ptr=ptr, nbr_idx=idx)


def _wall_state(p, gamma=1.4):
    """At rest (a wall state), density 1, the given pressures."""
    p = np.asarray(p, np.float64)
    return np.stack([np.ones_like(p), np.zeros_like(p), np.zeros_like(p), p / (gamma - 1.0)])


def _ellipse(n, a=0.5, b=0.06, xc=0.5):
    """Counter-clockwise, non-uniformly sampled ellipse with its exact
    outward (into the fluid) unit normals."""
    t = 2.0 * np.pi * np.arange(n) / n
    th = t + 0.4 * np.sin(t)  # monotone, smooth, periodic re-parametrisation
    x, y = xc + a * np.cos(th), b * np.sin(th)
    nx, ny = b * np.cos(th), a * np.sin(th)
    nr = np.hypot(nx, ny)
    return _ring(x, y, nx / nr, ny / nr), math.pi * a * b


@pytest.mark.parametrize("alpha", [0.0, 3.0, -7.5])
def test_forces_uniform_pressure_vanish(oracle_lib, alpha):
    n = 64
    t = 2.0 * np.pi * np.arange(n) / n
    c = _ring(0.5 + 0.5 * np.cos(t), 0.5 * np.sin(t), np.cos(t), np.sin(t))
    o = oracle.Oracle(c, oracle.params(mach=0.7, alpha_deg=alpha))
    cl, cd = o.forces(_wall_state(np.full(n, 1.0 / 1.4 + 0.3)))
    assert abs(cl) <= 1e-14 and abs(cd) <= 1e-14


@pytest.mark.parametrize("field", ["y", "x"])
@pytest.mark.parametrize("alpha", [0.0, 4.0])
def test_forces_linear_pressure_divergence_theorem(oracle_lib, field, alpha):
    """p = p_inf + s f with f = y (or x): F = -(0, s A) (or -(s A, 0));
    Cl = F.(-sin a, cos a)/q, Cd = F.(cos a, sin a)/q, q = rho_inf M^2/2.
    The polygon rule converges at second order in the spacing."""
    mach, s = 0.6, 0.25
    al = math.radians(alpha)
    qinf = 0.5 * mach * mach
    errs = []
    for n in (200, 400, 800):
        c, area = _ellipse(n)
        F = (0.0, -s * area) if field == "y" else (-s * area, 0.0)
        cl_x = (-F[0] * math.sin(al) + F[1] * math.cos(al)) / qinf
        cd_x = (F[0] * math.cos(al) + F[1] * math.sin(al)) / qinf
        o = oracle.Oracle(c, oracle.params(mach=mach, alpha_deg=alpha))
        f = c.y if field == "y" else c.x
        cl, cd = o.forces(_wall_state(1.0 / 1.4 + s * f))
        scale = s * area / qinf
        errs.append(max(abs(cl - cl_x), abs(cd - cd_x)) / scale)
    assert errs[-1] <= 2e-4, errs
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 <= e0 / e1 <= 4.5, errs


# -------------------------------------------------------------- limiter
def test_limiter_keeps_bounds_without_eps(oracle_lib):
    """eps = 0: q + phi delta lies in [qmin, qmax] for any q in the bounds and
    any increment (the limiter's defining property)."""
    rng = np.random.default_rng(3)
    for _ in range(4000):
        qmn, qmx = np.sort(rng.normal(size=2) * 10.0 ** rng.uniform(-3, 2))
        q = rng.uniform(qmn, qmx)
        delta = rng.choice([-1.0, 1.0]) * 10.0 ** rng.uniform(-4, 3) * (qmx - qmn)
        phi = oracle.venkat(delta, q, qmx, qmn, 0.0)
        v = q + phi * delta
        tol = 4e-16 * max(abs(qmn), abs(qmx))
        assert phi >= 0.0
        assert qmn - tol <= v <= qmx + tol, (q, qmn, qmx, delta, phi)


def test_limiter_limits_and_symmetry(oracle_lib):
    q, qmx, qmn = 0.3, 0.8, -0.1
    # phi -> 1 as the room to the bound grows against the increment
    for k in range(2, 9):
        d = 0.5 * 10.0 ** -k
        assert abs(oracle.venkat(d, q, qmx, qmn, 0.0) - 1.0) <= 4.0 * d / (qmx - q)
        assert abs(oracle.venkat(-d, q, qmx, qmn, 0.0) - 1.0) <= 4.0 * d / (q - qmn)
    # near a binding bound the limiter follows min(1, D/delta): phi/y -> 1 as
    # y = D/delta -> 0 (the smooth approximation of min(1, y) at its slope 1)
    for k in range(2, 7):
        y = 10.0 ** -k
        for d, qq in ((0.4, qmx - y * 0.4), (-0.4, qmn + y * 0.4)):
            yy = (qmx - qq) / d if d > 0 else (qmn - qq) / d
            phi = oracle.venkat(d, qq, qmx, qmn, 0.0)
            assert abs(phi / yy - 1.0) <= 2.0 * yy, (k, phi, yy)
    # phi -> 1 as eps grows
    for k in range(2, 10):
        eps2 = 10.0 ** k
        assert abs(oracle.venkat(2.0, q, qmx, qmn, eps2) - 1.0) <= 20.0 / eps2
    # a zero increment is not limited
    assert oracle.venkat(0.0, q, qmx, qmn, 0.0) == 1.0
    assert oracle.venkat(0.0, q, qmx, qmn, 1e-3) == 1.0
    # mirror symmetry: negating the increment, the value and the bounds
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b, qq = np.sort(rng.normal(size=3))[[0, 2, 1]]
        d, e2 = rng.normal(), 10.0 ** rng.uniform(-6, 1)
        assert oracle.venkat(d, qq, b, a, e2) == oracle.venkat(-d, -qq, -a, -b, e2)
    # increments towards a bound the point sits on are cut to zero
    assert oracle.venkat(0.2, qmx, qmx, qmn, 0.0) == 0.0
    assert oracle.venkat(-0.2, qmn, qmx, qmn, 0.0) == 0.0


def test_limiter_eps_homogeneous_degree_three(oracle_lib):
    for K, dx, dy in [(5.0, 0.01, -0.02), (0.3, 1.5, 0.25), (2.0, -3e-4, 1e-4)]:
        e = oracle.venkat_eps2(K, dx, dy)
        assert e > 0
        assert oracle.venkat_eps2(2 * K, dx, dy) == 8 * e
        assert oracle.venkat_eps2(K, 2 * dx, 2 * dy) == 8 * e
        assert oracle.venkat_eps2(0.5 * K, 4 * dx, 4 * dy) == 8 * e
    # it depends on the offset only through its length
    assert oracle.venkat_eps2(1.5, 3.0, 4.0) == oracle.venkat_eps2(1.5, 5.0, 0.0)
    assert oracle.venkat_eps2(1.5, 3.0, 4.0) == oracle.venkat_eps2(1.5, 0.0, -5.0)
    assert oracle.venkat_eps2(1.0, 3.0, 4.0) == 125.0


def _rough_q(c):
    rng = np.random.default_rng(11)
    U = smooth_state(c, amp=0.15)
    U[0] *= 1.0 + 0.05 * rng.uniform(-1, 1, c.n)
    U[3] *= 1.0 + 0.05 * rng.uniform(-1, 1, c.n)
    return U


def test_reconstruction_inside_bounds_as_eps_vanishes(oracle_lib):
    """With K -> 0 both modified states of every entry stay inside their own
    point's [qmin, qmax]; with K -> infinity the limiter lets the unlimited
    reconstruction through."""
    c = naca_ocloud(48, 16, jitter=0.1, seed=7)
    o = oracle.Oracle(c, oracle.params(limiter=1, venkat_k=1e-12))
    ev = o.evaluate(_rough_q(c))
    q, g, qmax, qmin = ev["q"], ev["g"], ev["qmax"], ev["qmin"]
    o_big = oracle.Oracle(c, oracle.params(limiter=1, venkat_k=1e9))
    o_off = oracle.Oracle(c, oracle.params(limiter=0))
    limited = 0
    for p in range(0, c.n, 7):
        for k in range(c.nbr_ptr[p], c.nbr_ptr[p + 1]):
            i = c.nbr_idx[k]
            qti, qt0 = o.modified_q(q, g, qmax, qmin, p, k)
            for qt, pt in ((qti, i), (qt0, p)):
                tol = 1e-15 * np.abs(q[:, pt]).max()
                assert np.all(qt >= qmin[:, pt] - tol) and np.all(qt <= qmax[:, pt] + tol)
            ui, u0 = o_off.modified_q(q, g, qmax, qmin, p, k)
            limited += int(np.any(ui != qti) or np.any(u0 != qt0))
            bi, b0 = o_big.modified_q(q, g, qmax, qmin, p, k)
            assert np.allclose(bi, ui, rtol=0, atol=1e-13) and np.allclose(b0, u0, rtol=0, atol=1e-13)
    assert limited > 100  # the field is rough enough for the limiter to act


@pytest.mark.parametrize("limiter", [0, 1])
def test_reconstruction_of_linear_fields(oracle_lib, limiter):
    """For a linear q field with its exact derivatives, eq. (28) shifts both
    states by -d/2 from their own point (d = P_i - P_0): q~_i is the field at
    the edge midpoint P_0 + d/2 and q~_0 the field at P_0 - d/2, so their
    difference is the full d.grad q.  The limiter leaves them untouched when
    its bounds are not binding (large K)."""
    c = naca_ocloud(48, 16, jitter=0.1, seed=9)
    o = oracle.Oracle(c, oracle.params(limiter=limiter, venkat_k=1e6))
    a = np.array([[-0.2, 0.3, 0.1], [0.1, -0.05, 1.2], [0.02, 0.04, -0.1], [0.01, -0.02, -2.8]])
    q = a[:, 0:1] * c.x + a[:, 1:2] * c.y + a[:, 2:3]
    g = np.concatenate([np.repeat(a[:, 0:1], c.n, 1), np.repeat(a[:, 1:2], c.n, 1)])
    qmax, qmin = q + 10.0, q - 10.0
    for p in range(0, c.n, 5):
        for k in range(c.nbr_ptr[p], c.nbr_ptr[p + 1]):
            i = c.nbr_idx[k]
            qti, qt0 = o.modified_q(q, g, qmax, qmin, p, k)
            mid = a[:, 0] * 0.5 * (c.x[p] + c.x[i]) + a[:, 1] * 0.5 * (c.y[p] + c.y[i]) + a[:, 2]
            back = (a[:, 0] * 0.5 * (3 * c.x[p] - c.x[i]) + a[:, 1] * 0.5 * (3 * c.y[p] - c.y[i])
                    + a[:, 2])
            assert np.allclose(qti, mid, rtol=0, atol=1e-14)
            assert np.allclose(qt0, back, rtol=0, atol=1e-14)
