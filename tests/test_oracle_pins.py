"""Pins of the FP64 oracle against what the paper and the mathematics fix,
independently of the oracle's own formulas.

  split fluxes      : brute-force quadrature of the half-range moments of the
                      Maxwellian (sec. 2 eqs. (4)-(9)); G+ + G- = Euler flux
                      (eqs. (1)-(2)); limits
  q-variables       : U -> q -> U round trip; q equals the gradient of the
                      entropy -rho s/(gamma-1) up to a constant (uniqueness of
                      the U <-> q map, sec. 2.1)
  least squares     : exact derivatives of linear fields (eq. (11));
                      k-exactness of the converged inner iterations for
                      quadratics (sec. 2.1, eqs. (23), (29))
  flux residual     : freestream preservation on any cloud; second-order
                      consistency with the exact flux divergence (eq. (1));
                      rotation invariance; mirror symmetry
  Runge-Kutta       : stability polynomial 1 + z + z^2/2 + z^3/6 + z^4/48
  wall condition    : tangency after every iteration
  restart           : 50 + 50 iterations == 100 iterations, bitwise
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from cloudgen import naca_ocloud, random_cloud, rotate_cloud
from tests._common import GAMMA, normwise_rel, smooth_state


# ---------------------------------------------------------------- fluxes
def _quadrature_split_flux(prim, e, sign, gamma=GAMMA, dps=30):
    """<Psi, v_e^{+-} F> by quadrature.  F = (rho/I0)(beta/pi)
    exp(-beta|v-u|^2 - I/I0), I0 = (2-gamma)/(2 beta (gamma-1)),
    Psi = (1, v1, v2, I + |v|^2/2).  The I integral is exact (moments of an
    exponential), v_perp by 20-point Gauss-Hermite (exact for the polynomial
    degrees present), v_e over the half line by tanh-sinh quadrature."""
    mp.mp.dps = dps
    rho, u1, u2, p = (mp.mpf(float(v)) for v in prim)
    beta = rho / (2 * p)
    g = mp.mpf(gamma)
    I0 = (2 - g) / (2 * beta * (g - 1))
    ex, ey = mp.mpf(float(e[0])), mp.mpf(float(e[1]))
    px, py = -ey, ex  # perpendicular unit vector
    ue = u1 * ex + u2 * ey
    up = u1 * px + u2 * py
    xs, ws = np.polynomial.hermite.hermgauss(20)
    nodes = [(up + mp.mpf(float(xk)) / mp.sqrt(beta), mp.mpf(float(wk)) / mp.sqrt(beta))
             for xk, wk in zip(xs, ws)]

    def integrand(ve, comp):
        tot = mp.mpf(0)
        for vp, w in nodes:
            v1 = ve * ex + vp * px
            v2 = ve * ey + vp * py
            psi = (1, v1, v2, I0 + (v1 * v1 + v2 * v2) / 2)[comp]
            tot += w * psi
        return ve * tot * rho * (beta / mp.pi) * mp.exp(-beta * (ve - ue) ** 2)

    lo, hi = (0, mp.inf) if sign > 0 else (-mp.inf, 0)
    return np.array([float(mp.quad(lambda v: integrand(v, c), [lo, hi])) for c in range(4)])


STATES = [((1.0, 0.6, 0.1, 1 / 1.4), (1.0, 0.0)),
          ((0.8, -0.3, 0.5, 0.5), (0.6, 0.8)),
          ((1.3, 2.0, -0.4, 0.9), (0.0, 1.0)),   # supersonic along e
          ((0.7, 0.0, 0.0, 0.6), (np.sqrt(0.5), -np.sqrt(0.5)))]


@pytest.mark.parametrize("prim,e", STATES)
@pytest.mark.parametrize("sign", [1, -1])
def test_split_flux_vs_quadrature(oracle_lib, prim, e, sign):
    G = oracle.split_flux(prim, e, sign)
    Gq = _quadrature_split_flux(prim, e, sign)
    scale = np.abs(Gq).max()
    assert np.abs(G - Gq).max() <= 1e-13 * scale, (G, Gq)


@pytest.mark.parametrize("prim,e", STATES)
def test_split_fluxes_sum_to_euler_flux(oracle_lib, prim, e):
    rho, u1, u2, p = prim
    ue = u1 * e[0] + u2 * e[1]
    rhoe = p / (GAMMA - 1) + 0.5 * rho * (u1 * u1 + u2 * u2)
    euler = np.array([rho * ue, rho * u1 * ue + p * e[0], rho * u2 * ue + p * e[1],
                      (p + rhoe) * ue])
    tot = oracle.split_flux(prim, e, 1) + oracle.split_flux(prim, e, -1)
    assert np.abs(tot - euler).max() <= 4e-16 * np.abs(euler).max() + 1e-300


def test_split_flux_limits(oracle_lib):
    # at rest the + mass flux is the one-sided thermal flux rho / (2 sqrt(pi beta))
    rho, p = 1.2, 0.7
    beta = rho / (2 * p)
    G = oracle.split_flux((rho, 0.0, 0.0, p), (1.0, 0.0), 1)
    assert abs(G[0] - rho / (2 * np.sqrt(np.pi * beta))) <= 1e-16
    # far supersonic along +e: nothing travels backwards
    Gm = oracle.split_flux((1.0, 40.0, 0.0, 0.1), (1.0, 0.0), -1)
    assert np.all(Gm == 0.0)


# ---------------------------------------------------------------- q variables
def test_q_roundtrip_and_entropy_gradient(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(50):
        prim = np.array([rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2),
                         rng.uniform(0.1, 3)])
        U = oracle.prim_to_u(prim)
        q = oracle.prim_to_q(oracle.u_to_prim(U))
        U2 = oracle.prim_to_u(oracle.q_to_prim(q))
        assert np.abs(U2 - U).max() <= 1e-14 * np.abs(U).max()
        # q = d eta / dU + const, eta = -rho s/(gamma-1), s = ln(p / rho^gamma)
        mp.mp.dps = 40
        Um = [mp.mpf(float(v)) for v in U]

        def eta(*u):
            r, m1, m2, E = u
            pr = (GAMMA - 1) * (E - (m1 * m1 + m2 * m2) / (2 * r))
            return -r * (mp.log(pr) - GAMMA * mp.log(r)) / (GAMMA - 1)

        grad = [mp.diff(lambda t, k=k: eta(*[Um[j] + (t if j == k else 0) for j in range(4)]), 0)
                for k in range(4)]
        const = -(GAMMA + np.log(2.0)) / (GAMMA - 1)
        expect = np.array([float(grad[0]) + const, float(grad[1]), float(grad[2]),
                           float(grad[3])])
        assert np.abs(q - expect).max() <= 1e-13 * max(1.0, np.abs(expect).max())


# ---------------------------------------------------------------- least squares
@pytest.mark.parametrize("which", ["small", "jitter", "random"])
@pytest.mark.parametrize("n_inner", [0, 3, 10])
def test_ls_exact_for_linear_fields(oracle_lib, which, n_inner):
    c = {"small": lambda: naca_ocloud(48, 16),
         "jitter": lambda: naca_ocloud(40, 20, jitter=0.1, seed=5),
         "random": lambda: random_cloud(300, seed=3)}[which]()
    o = oracle.Oracle(c)
    A = np.array([[0.3, -1.2, 0.7], [1.1, 0.4, -0.2], [-0.5, 2.0, 0.9], [-2.0, 0.1, 0.3]])
    q = A[:, :1] + A[:, 1:2] * c.x + A[:, 2:3] * c.y
    g, qmax, qmin = o.q_derivatives(q, n_inner)
    exact = np.concatenate([np.repeat(A[:, 1:2], c.n, 1), np.repeat(A[:, 2:3], c.n, 1)])
    assert np.abs(g - exact).max() <= 1e-12 * np.abs(A).max()
    # bounds contain the point's own value
    assert np.all(qmax >= q) and np.all(qmin <= q)


def test_inner_iterations_k_exact_for_quadratics(oracle_lib):
    """The converged defect-correction derivatives are exact for
    polynomials of degree <= 2 (k-exactness), and the error falls with the
    number of inner iterations."""
    c = naca_ocloud(40, 16, jitter=0.1, seed=9)
    o = oracle.Oracle(c)
    x, y = c.x, c.y
    q = np.stack([0.3 + 0.2 * x - 0.1 * y + 0.05 * x * x + 0.07 * x * y - 0.03 * y * y,
                  0.1 * x + 0.2 * y * y, -0.3 * x * y + 0.1 * y, 0.2 * x * x - 0.1 * y])
    gx = np.stack([0.2 + 0.1 * x + 0.07 * y, 0.1 + 0 * x, -0.3 * y, 0.4 * x])
    gy = np.stack([-0.1 + 0.07 * x - 0.06 * y, 0.4 * y, -0.3 * x + 0.1, -0.1 + 0 * x])
    exact = np.concatenate([gx, gy])
    errs = []
    for k in (0, 3, 10, 30, 300):
        g, _, _ = o.q_derivatives(q, k)
        errs.append(np.abs(g - exact).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[-1] <= 1e-9


# ---------------------------------------------------------------- residual
@pytest.mark.parametrize("limiter", [0, 1])
def test_freestream_residual_is_exactly_zero(oracle_lib, limiter):
    for c in (random_cloud(300, seed=21), naca_ocloud(48, 16, jitter=0.1, seed=4)):
        o = oracle.Oracle(c, oracle.params(limiter=limiter, mach=0.7, alpha_deg=-3.0))
        o.require_valid()
        U = o.freestream(project_wall=False)
        ev = o.evaluate(U)
        assert np.count_nonzero(ev["R"]) == 0
    # without wall points (whose projection changes a raw freestream) the
    # state does not move at all
    c = random_cloud(300, seed=22, wall_fraction=0.0)
    o = oracle.Oracle(c, oracle.params(limiter=limiter, mach=0.7, alpha_deg=-3.0))
    U = o.freestream(project_wall=False)
    U2, _ = o.run(U, 3)
    np.testing.assert_array_equal(U2, U)


def _periodic_lattice(n, h, jitter, seed):
    """Jittered square lattice of (n x n) points with spacing h around the
    origin, 5 x 5 box connectivity, global frame; the outer two rings are
    outer points (they only supply neighbours)."""
    from cloudgen import Cloud, uniform
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i, j = i.reshape(-1), j.reshape(-1)
    r = uniform(seed, 2 * n * n, -jitter, jitter).reshape(2, -1)
    x = (i - (n - 1) / 2 + r[0]) * h
    y = (j - (n - 1) / 2 + r[1]) * h
    kind = np.where((i < 2) | (j < 2) | (i >= n - 2) | (j >= n - 2), 2, 0).astype(np.uint8)
    rows, cols = [], []
    for p in range(n * n):
        for b in range(-2, 3):
            for a in range(-2, 3):
                if a == 0 and b == 0:
                    continue
                ii, jj = i[p] + a, j[p] + b
                if 0 <= ii < n and 0 <= jj < n:
                    rows.append(p)
                    cols.append(jj * n + ii)
    rows, cols = np.array(rows), np.array(cols)
    ptr = np.zeros(n * n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=n * n), out=ptr[1:])
    return Cloud(x=x, y=y, nx=np.zeros(n * n), ny=np.ones(n * n), kind=kind, nbr_ptr=ptr,
                 nbr_idx=cols.astype(np.int32))


def _exact_divergence(x, y, mach=0.6, amp=0.08):
    """d(Gx)/dx + d(Gy)/dy of the smooth field below, by complex-step
    differentiation of the exact Euler fluxes."""
    def prim(xx, yy):
        rho = 1.0 + amp * np.sin(2 * xx + 0.3) * np.cos(1.5 * yy)
        u1 = mach * (1.0 + amp * np.cos(xx - 2 * yy))
        u2 = 0.2 * mach + amp * mach * np.sin(1.5 * xx + yy)
        p = (1 / GAMMA) * (1.0 + amp * np.cos(xx + 0.7 * yy))
        return rho, u1, u2, p

    def flux(xx, yy):
        rho, u1, u2, p = prim(xx, yy)
        rhoe = p / (GAMMA - 1) + 0.5 * rho * (u1 * u1 + u2 * u2)
        gx = [rho * u1, rho * u1 * u1 + p, rho * u1 * u2, (p + rhoe) * u1]
        gy = [rho * u2, rho * u1 * u2, rho * u2 * u2 + p, (p + rhoe) * u2]
        return np.array(gx), np.array(gy)

    hcs = 1e-30
    gx, _ = flux(x + 1j * hcs, y)
    _, gy = flux(x, y + 1j * hcs)
    div = (gx.imag + gy.imag) / hcs
    rho, u1, u2, p = prim(x, y)
    U = np.stack([rho, rho * u1, rho * u2, p / (GAMMA - 1) + 0.5 * rho * (u1 * u1 + u2 * u2)])
    return U, div


def _consistency_errors(n_inner, levels=((24, 0.08), (48, 0.04)), order=2):
    errs = []
    for n, h in levels:
        c = _periodic_lattice(n, h, 0.15, seed=7)
        o = oracle.Oracle(c, oracle.params(limiter=0, n_inner=n_inner, order=order))
        o.require_valid()
        U, div = _exact_divergence(c.x, c.y)
        R = o.evaluate(U)["R"]
        core = (np.abs(c.x) < 0.3) & (np.abs(c.y) < 0.3)
        errs.append(np.abs(R[:, core] - div[:, core]).max() / np.abs(div[:, core]).max())
    return errs


def test_residual_consistent_second_order(oracle_lib):
    """On jittered lattices the residual R converges to the exact flux
    divergence of eq. (1): at second order once the inner iterations of
    eq. (29) have converged (the defect correction of sec. 2.1), at first
    order with none (q~ built from the first-order gradient)."""
    e2 = _consistency_errors(30)
    assert e2[0] < 0.03
    assert e2[0] / e2[1] > 3.6, e2
    e1 = _consistency_errors(0)
    assert 1.7 < e1[0] / e1[1] < 2.6, e1


def test_first_order_mode_consistent_first_order(oracle_lib):
    """First-order LSKUM (the split-flux derivatives of eqs. (12)-(14) applied
    to the fluxes of q itself, no modified q): the residual converges to the
    flux divergence at first order, and no q-derivative enters it."""
    e = _consistency_errors(0, order=1)
    assert e[0] < 0.3  # 0.24 at h = 0.08, 0.127 at 0.04, 0.066 at 0.02
    assert 1.7 < e[0] / e[1] < 2.3, e
    c = _periodic_lattice(24, 0.08, 0.15, seed=7)
    U, _ = _exact_divergence(c.x, c.y)
    R0 = oracle.Oracle(c, oracle.params(n_inner=0, order=1)).evaluate(U)["R"]
    R3 = oracle.Oracle(c, oracle.params(n_inner=3, order=1)).evaluate(U)["R"]
    np.testing.assert_array_equal(R0, R3)


def test_rotation_invariance(oracle_lib):
    c = naca_ocloud(40, 16, jitter=0.1, seed=8)
    th = np.radians(30.0)
    cr = rotate_cloud(c, th)
    o = oracle.Oracle(c, oracle.params(alpha_deg=2.0))
    orr = oracle.Oracle(cr, oracle.params(alpha_deg=32.0))
    assert np.array_equal(o.flag, orr.flag)
    U = smooth_state(c)
    Ur = U.copy()
    Ur[1] = np.cos(th) * U[1] - np.sin(th) * U[2]
    Ur[2] = np.sin(th) * U[1] + np.cos(th) * U[2]
    R = o.evaluate(U)["R"]
    Rr = orr.evaluate(Ur)["R"]
    Rback = Rr.copy()
    Rback[1] = np.cos(th) * Rr[1] + np.sin(th) * Rr[2]
    Rback[2] = -np.sin(th) * Rr[1] + np.cos(th) * Rr[2]
    assert np.abs(Rback - R).max() <= 1e-12 * np.abs(R).max()


def test_mirror_symmetry_zero_incidence(oracle_lib):
    """Symmetric airfoil at zero incidence on a mirror-exact cloud: the flow
    stays symmetric and the lift vanishes."""
    ns, nr = 48, 16
    c = naca_ocloud(ns, nr)
    o = oracle.Oracle(c, oracle.params(mach=0.63, alpha_deg=0.0))
    U, _ = o.run(o.freestream(), 300)
    m = ns // 2
    i = np.arange(1, m)
    X = lambda a: a.reshape(nr, ns)
    rho = X(U[0])
    assert np.abs(rho[:, i] - rho[:, ns - i]).max() <= 1e-10
    assert np.abs(X(U[2])[:, i] + X(U[2])[:, ns - i]).max() <= 1e-10
    cl, cd = o.forces(U)
    assert abs(cl) <= 1e-10


# ---------------------------------------------------------------- time march
def test_rk_stability_polynomial(oracle_lib):
    lam = -0.7 + 0.3j
    for dt in (0.05, 0.2, 0.8):
        z = lam * dt
        u0 = 1.0 + 0.5j

        def stage(rk, un, u):
            re = oracle.rk_stage(rk, [un.real], [u.real], [-(lam * u).real], [dt])[0]
            im = oracle.rk_stage(rk, [un.imag], [u.imag], [-(lam * u).imag], [dt])[0]
            return re + 1j * im

        u1 = stage(1, u0, u0)
        u2 = stage(2, u0, u1)
        u3 = stage(3, u0, u2)
        u4 = stage(4, u0, u3)
        poly = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 48
        assert abs(u4 - poly * u0) <= 1e-15 * abs(u0) * 4


def test_wall_tangency_and_restart(oracle_lib):
    c = naca_ocloud(48, 16)
    o = oracle.Oracle(c)
    U0 = o.freestream()
    U50, h1 = o.run(U0, 50)
    wall = c.kind == 1
    mn = U50[1, wall] * c.nx[wall] + U50[2, wall] * c.ny[wall]
    mm = np.hypot(U50[1, wall], U50[2, wall])
    assert np.all(np.abs(mn) <= 1e-14 * mm + 1e-300)
    U100, _ = o.run(U0, 100)
    Ur, h2 = o.run(U50, 50)
    np.testing.assert_array_equal(Ur, U100)
    assert h1[0, 0] > 0


def test_singular_stencil_is_rejected(oracle_lib):
    from cloudgen import Cloud
    n = 6
    line = Cloud(x=np.arange(n, dtype=float), y=np.zeros(n), nx=np.zeros(n), ny=np.ones(n),
                 kind=np.zeros(n, np.uint8), nbr_ptr=np.arange(0, 5 * n + 1, 5, dtype=np.int32),
                 nbr_idx=np.array([j for i in range(n) for j in range(n) if j != i], np.int32))
    o = oracle.Oracle(line)
    assert o.classify_status == oracle.ESINGULAR


# ---------------------------------------------------------------- brute force
def _five_point_bruteforce(c, U, limiter, n_inner=3, K=5.0, dps=30, order=2):
    """Independent evaluation of the stage operator at P0 of the five-point
    cloud in 30-digit arithmetic: q from eq. (26); q-derivatives by QR least
    squares of eq. (11) and of the defect-corrected differences of eq. (29)
    (Jacobi); q~ of eq. (28) with the Venkatakrishnan factor when asked;
    split fluxes by quadrature of the Maxwellian's half-range moments; each
    split stencil of P0 holds exactly two points, so its derivative of
    eq. (13) is the exact solution of a 2x2 interpolation system."""
    mp.mp.dps = dps
    n = c.n
    X = [mp.mpf(float(v)) for v in c.x]
    Y = [mp.mpf(float(v)) for v in c.y]
    g_ = mp.mpf(GAMMA)
    q = []
    for p in range(n):
        rho = mp.mpf(float(U[0, p]))
        u1, u2 = mp.mpf(float(U[1, p])) / rho, mp.mpf(float(U[2, p])) / rho
        pr = (g_ - 1) * (mp.mpf(float(U[3, p])) - rho * (u1 ** 2 + u2 ** 2) / 2)
        beta = rho / (2 * pr)
        q.append([mp.log(rho) + mp.log(beta) / (g_ - 1) - beta * (u1 ** 2 + u2 ** 2),
                  2 * beta * u1, 2 * beta * u2, -2 * beta])
    nbrs = [[int(i) for i in c.nbr_idx[c.nbr_ptr[p]:c.nbr_ptr[p + 1]]] for p in range(n)]

    def ls(p, rhs):
        A = mp.matrix([[X[i] - X[p], Y[i] - Y[p]] for i in nbrs[p]])
        sol, _ = mp.qr_solve(A, mp.matrix(rhs))
        return sol[0], sol[1]

    g = [[ls(p, [q[i][r] - q[p][r] for i in nbrs[p]]) for r in range(4)] for p in range(n)]
    for _ in range(n_inner):
        g = [[ls(p, [q[i][r] - q[p][r] - ((X[i] - X[p]) * (g[i][r][0] - g[p][r][0]) +
                                           (Y[i] - Y[p]) * (g[i][r][1] - g[p][r][1])) / 2
                     for i in nbrs[p]]) for r in range(4)] for p in range(n)]
    qmax = [[max([q[p][r]] + [q[i][r] for i in nbrs[p]]) for r in range(4)] for p in range(n)]
    qmin = [[min([q[p][r]] + [q[i][r] for i in nbrs[p]]) for r in range(4)] for p in range(n)]

    def recon(p, dx, dy, r, eps2):
        if order == 1:
            return q[p][r]
        d = -(dx * g[p][r][0] + dy * g[p][r][1]) / 2
        if not limiter:
            return q[p][r] + d
        D = (qmax[p][r] - q[p][r]) if d > 0 else (qmin[p][r] - q[p][r])
        den = D * D + 2 * d * d + d * D + eps2
        phi = 1 if den == 0 else ((D * D + eps2) + 2 * d * D) / den
        return q[p][r] + phi * d

    def prim_of(qt):
        beta = -qt[3] / 2
        u1, u2 = qt[1] / (2 * beta), qt[2] / (2 * beta)
        rho = mp.exp(qt[0] - mp.log(beta) / (g_ - 1) + beta * (u1 ** 2 + u2 ** 2))
        return (rho, u1, u2, rho / (2 * beta))

    p0 = 0
    ex_n, ey_n = float(c.nx[p0]), float(c.ny[p0])
    frames = {"s": (ey_n, -ex_n), "n": (ex_n, ey_n)}
    Gpair = {}
    for i in nbrs[p0]:
        dx, dy = X[i] - X[p0], Y[i] - Y[p0]
        eps2 = (K * mp.sqrt(dx * dx + dy * dy)) ** 3
        qti = [recon(i, dx, dy, r, eps2) for r in range(4)]
        qt0 = [recon(p0, dx, dy, r, eps2) for r in range(4)]
        Gpair[i] = (prim_of(qti), prim_of(qt0), dx, dy)
    R = np.zeros(4)
    parts = []
    for axis in ("s", "n"):
        e = frames[axis]
        es = mp.mpf(e[0]), mp.mpf(e[1])
        other = frames["n" if axis == "s" else "s"]
        for sign in (1, -1):
            members = []
            for i, (pi, p0s, dx, dy) in Gpair.items():
                da = dx * es[0] + dy * es[1]
                if (da < 0) == (sign > 0):
                    members.append(i)
            assert len(members) == 2
            rows, rhs = [], []
            for i in members:
                pi, p0s, dx, dy = Gpair[i]
                ds = dx * mp.mpf(frames["s"][0]) + dy * mp.mpf(frames["s"][1])
                dn = dx * mp.mpf(frames["n"][0]) + dy * mp.mpf(frames["n"][1])
                Gi = _quadrature_split_flux([float(v) for v in pi], e, sign, dps=dps)
                G0 = _quadrature_split_flux([float(v) for v in p0s], e, sign, dps=dps)
                rows.append([ds, dn])
                rhs.append(Gi - G0)
            M = mp.matrix(rows)
            d = np.zeros(4)
            for r in range(4):
                sol = mp.lu_solve(M, mp.matrix([rhs[0][r], rhs[1][r]]))
                d[r] = float(sol[0] if axis == "s" else sol[1])
            parts.append(d)
            R += d
    gout = np.array([[float(g[p][r][0]) for p in range(n)] for r in range(4)] +
                    [[float(g[p][r][1]) for p in range(n)] for r in range(4)])
    return gout, R, np.array(parts)


@pytest.mark.parametrize("limiter,order", [(0, 2), (1, 2), (0, 1)])
def test_five_point_bruteforce(oracle_lib, limiter, order):
    """Five points, complete connectivity, global frame; P1..P4 supply
    neighbours only.  Oracle g (all points) and R (P0) against the
    independent 30-digit evaluation above (second order with and without
    the limiter, and first order)."""
    from cloudgen import five_point_cloud
    c = five_point_cloud(0.05)
    c.kind[1:] = 2
    o = oracle.Oracle(c, oracle.params(limiter=limiter, n_inner=3, venkat_k=5.0, order=order))
    o.require_valid()
    U = smooth_state(c, amp=0.3)
    ev = o.evaluate(U)
    g_bf, R_bf, parts = _five_point_bruteforce(c, U, limiter, order=order)
    assert np.abs(ev["g"] - g_bf).max() <= 1e-13 * np.abs(g_bf).max()
    scale = np.abs(parts).max()
    assert np.abs(ev["R"][:, 0] - R_bf).max() <= 1e-13 * scale, (ev["R"][:, 0], R_bf)
