"""Learned warm start through the C ABI: features -> network -> state, the
per-case comparison of the first residual with the freestream's, and the
fallback."""
import numpy as np
import pytest

from cloudgen import naca_ocloud
from tests._common import normwise_rel

pytestmark = pytest.mark.gpu

GAMMA = 1.4
CASES = [dict(tau=0.12, mach=0.63, alpha=2.0), dict(tau=0.10, mach=0.5, alpha=-1.0)]


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2108_07031_amd import qlskum
    return torch, qlskum


@pytest.fixture(scope="module")
def clouds():
    return [naca_ocloud(48, 16, tau=c["tau"]) for c in CASES]


def _say(msg):
    print(msg, flush=True)


def _batch(ql, clouds, **prm):
    s = ql.Solver(limiter=1, **prm)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    return s, offs


def _features(s, clouds):
    """(x, y, log wall distance, M, alpha, tau) per point, caller order."""
    d = s.wall_distance()
    cols = []
    for cl, c in zip(clouds, CASES):
        cols.append(np.stack([cl.x, cl.y, np.zeros(cl.n), np.full(cl.n, c["mach"]),
                              np.full(cl.n, c["alpha"]), np.full(cl.n, c["tau"])], axis=1))
    F = np.concatenate(cols)
    F[:, 2] = np.log(d + 1e-3)
    return F


def _prims(U):
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    p = (GAMMA - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return np.stack([rho, u, v, p], axis=1)


def test_wall_distance(env, clouds):
    torch, ql = env
    _say("wall distance")
    s, offs = _batch(ql, clouds)
    d = s.wall_distance()
    for i, cl in enumerate(clouds):
        w = np.flatnonzero(cl.kind == 1)
        dd = d[offs[i]:offs[i + 1]]
        ref = np.sqrt(((cl.x[:, None] - cl.x[w][None, :]) ** 2 +
                       (cl.y[:, None] - cl.y[w][None, :]) ** 2).min(axis=1))
        np.testing.assert_allclose(dd, ref, rtol=1e-15, atol=0)
        assert np.all(dd[w] == 0.0)
    s.close()


def test_garbage_network_falls_back(env, clouds):
    torch, ql = env
    _say("garbage network")
    s, _ = _batch(ql, clouds)
    s.init_freestream()
    U_cold = s.fetch_state()
    m = ql.Mlp([6, 16, 4], max_batch=4096)
    rng = np.random.default_rng(3)
    m.set_weights(100.0 * rng.normal(size=m.num_params))
    F = _features(s, clouds)
    rc, rw, used = s.warm_start(m, torch.tensor(F, dtype=torch.float32, device="cuda"),
                                [1, 0, 0, 0.7, 1, 1, 1, 1])
    _say(f"  cold {rc[:, 0]}, warm {rw[:, 0]}, used {used}")
    assert not used.any()
    np.testing.assert_array_equal(s.fetch_state(), U_cold)
    m.close()
    s.close()


# training conditions around the held-out ones (the network interpolates
# between flow conditions; it is trained on converged solutions of these)
TRAIN = [dict(tau=0.12, mach=0.63, alpha=2.0), dict(tau=0.10, mach=0.5, alpha=-1.0),
         dict(tau=0.11, mach=0.55, alpha=0.5), dict(tau=0.13, mach=0.6, alpha=-0.5),
         dict(tau=0.10, mach=0.65, alpha=1.5), dict(tau=0.12, mach=0.52, alpha=-2.0)]
HELD = [dict(tau=0.115, mach=0.58, alpha=0.8), dict(tau=0.105, mach=0.56, alpha=-0.6)]


def test_trained_network_converges_sooner(env):
    """A network trained on converged solutions of six conditions starts two
    held-out conditions (other Mach number, incidence and thickness, other
    clouds): the warm start is taken, its state is the warm-start map of the
    network's outputs point by point (the FP64 reference oracle.warm; 1e-14
    normwise per component), its first residual is below the freestream's,
    and it reaches the residual drop in fewer iterations than the cold
    start."""
    import oracle.warm as ow
    torch, ql = env
    _say("trained network, held-out conditions")
    drop = 1e-3
    cl_train = [naca_ocloud(48, 16, tau=c["tau"]) for c in TRAIN]
    cl_held = [naca_ocloud(48, 16, tau=c["tau"]) for c in HELD]

    def batch(clouds, conds):
        s = ql.Solver(limiter=1)
        offs = s.upload_batch(clouds, [c["mach"] for c in conds], [c["alpha"] for c in conds])
        return s, offs

    def features(s, clouds, conds):
        d = s.wall_distance()
        F = np.concatenate([np.stack([cl.x, cl.y, np.zeros(cl.n), np.full(cl.n, c["mach"]),
                                      np.full(cl.n, c["alpha"]), np.full(cl.n, c["tau"])], axis=1)
                            for cl, c in zip(clouds, conds)])
        F[:, 2] = np.log(d + 1e-3)
        return F

    s, _ = batch(cl_train, TRAIN)
    s.init_freestream()
    s.batch_run(drop, 20000, check_every=200)
    assert list(s.batch_status()) == [ql.QL_OK] * len(TRAIN)
    U = s.fetch_state()
    F = features(s, cl_train, TRAIN)
    s.close()
    kind = np.concatenate([cl.kind for cl in cl_train])
    P = _prims(U)
    fm, fs = F.mean(axis=0), F.std(axis=0) + 1e-12
    pm, ps = P.mean(axis=0), P.std(axis=0) + 1e-12
    keep = kind != 2
    Xt = torch.tensor((F[keep] - fm) / fs, dtype=torch.float32, device="cuda")
    Yt = torch.tensor((P[keep] - pm) / ps, dtype=torch.float32, device="cuda")
    widths = [6, 64, 64, 64, 4]
    rng = np.random.default_rng(11)
    w0 = np.concatenate([np.concatenate([rng.normal(0, np.sqrt(1.0 / a), a * b),
                                         np.zeros(b)]) for a, b in zip(widths[:-1], widths[1:])])
    m = ql.Mlp(widths, max_batch=Xt.shape[0])
    m.set_weights(w0)
    for t in range(3000):
        loss = m.train_step(Xt, Yt, 3e-3 if t < 2200 else 1e-3, want_loss=(t % 500 == 499))
        if t % 500 == 499:
            _say(f"  step {t + 1}: loss {loss:.3e}")
    # held-out conditions: cold, then warm
    sc, _ = batch(cl_held, HELD)
    sc.init_freestream()
    iters_cold, _ = sc.batch_run(drop, 20000, check_every=200)
    Fh = features(sc, cl_held, HELD)
    sc.close()
    sw, offs = batch(cl_held, HELD)
    X = torch.tensor((Fh - fm) / fs, dtype=torch.float32, device="cuda")
    scale = np.concatenate([pm, ps]).astype(np.float32)
    rc, rw, used = sw.warm_start(m, X, scale)
    Uw = sw.fetch_state()
    Y = m.forward(X).cpu().numpy()
    for i, (cl, c) in enumerate(zip(cl_held, HELD)):
        lo, hi = int(offs[i]), int(offs[i + 1])
        ref = ow.warm_state(Y[lo:hi], scale[:4], scale[4:], 0.05, cl.kind, cl.nx, cl.ny,
                            c["mach"], c["alpha"])
        err = normwise_rel(Uw[:, lo:hi], ref)
        _say(f"  case {i}: warm state vs reference map {err.max():.2e}")
        assert np.all(err <= 1e-14), (i, err)
    iters_warm, _ = sw.batch_run(drop, 20000, check_every=200, ref=rc[:, 0])
    _say(f"  R(1) cold {rc[:, 0]}, warm {rw[:, 0]}; iterations cold {iters_cold}, "
         f"warm {iters_warm}")
    assert used.all()
    assert np.all(rw[:, 0] < rc[:, 0])
    assert np.all(iters_warm < iters_cold)
    m.close()
    sw.close()
