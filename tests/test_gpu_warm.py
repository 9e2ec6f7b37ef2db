"""Learned warm start through the C ABI: features -> network -> state, the
per-case comparison of the first residual with the freestream's, and the
fallback."""
import numpy as np
import pytest

from cloudgen import naca_ocloud

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


def test_trained_network_converges_sooner(env, clouds):
    torch, ql = env
    _say("trained network")
    drop = 1e-3
    s, offs = _batch(ql, clouds)
    s.init_freestream()
    iters_cold, _ = s.batch_run(drop, 20000, check_every=200)
    U = s.fetch_state()
    F = _features(s, clouds)
    kind = np.concatenate([cl.kind for cl in clouds])
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
    for t in range(2000):
        loss = m.train_step(Xt, Yt, 3e-3 if t < 1500 else 1e-3, want_loss=(t % 500 == 499))
        if t % 500 == 499:
            _say(f"  step {t + 1}: loss {loss:.3e}")
    s2, _ = _batch(ql, clouds)
    X = torch.tensor((F - fm) / fs, dtype=torch.float32, device="cuda")
    rc, rw, used = s2.warm_start(m, X, np.concatenate([pm, ps]))
    iters_warm, _ = s2.batch_run(drop, 20000, check_every=200, ref=rc[:, 0])
    _say(f"  R(1) cold {rc[:, 0]}, warm {rw[:, 0]}; iterations cold {iters_cold}, "
         f"warm {iters_warm}")
    assert used.all()
    assert np.all(rw[:, 0] < rc[:, 0])
    assert np.all(iters_warm < iters_cold)
    m.close()
    s.close()
    s2.close()
