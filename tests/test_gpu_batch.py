"""Batched form: several independent clouds with their own flow conditions
advanced by the same launches.

Each point's arithmetic does not depend on which other cases share the
launch, and each case's residual norm is summed over chunks that start at
the case's first point, so a batched run reproduces the solo runs bit for
bit (FP64 and mixed).  Graph replay runs the same kernels as eager launches
and must match them bit for bit; a retired case stops at exactly the
iteration its solo residual history reaches the drop.
"""
import numpy as np
import pytest

from cloudgen import naca_ocloud

pytestmark = pytest.mark.gpu

CASES = [dict(ns=48, nr=16, tau=0.12, jitter=0.0, mach=0.63, alpha=2.0),
         dict(ns=64, nr=24, tau=0.10, jitter=0.1, mach=0.5, alpha=-1.5),
         dict(ns=40, nr=20, tau=0.15, jitter=0.05, mach=0.75, alpha=4.0)]


@pytest.fixture(scope="module")
def ql():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2108_07031_amd import qlskum
    return qlskum


@pytest.fixture(scope="module")
def clouds():
    return [naca_ocloud(c["ns"], c["nr"], tau=c["tau"], jitter=c["jitter"], seed=7 + i)
            for i, c in enumerate(CASES)]


def _say(msg):
    print(msg, flush=True)


def _solo(ql, cloud, case, n_iter, **prm):
    s = ql.Solver(cloud, mach=case["mach"], alpha_deg=case["alpha"], **prm)
    s.init_freestream()
    h = s.step(n_iter)
    U = s.fetch_state()
    s.close()
    return U, h


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_solo(ql, clouds, precision):
    _say(f"batched vs solo precision={precision}")
    prm = dict(limiter=1, precision=precision)
    s = ql.Solver(**prm)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    s.init_freestream()
    hb = s.step(30)
    Ub = s.fetch_state()
    assert hb.shape == (30, len(CASES), 4)
    for i, (cl, case) in enumerate(zip(clouds, CASES)):
        U, h = _solo(ql, cl, case, 30, **prm)
        np.testing.assert_array_equal(Ub[:, offs[i]:offs[i + 1]], U)
        np.testing.assert_array_equal(hb[:, i], h)
    clb, cdb = s.batch_forces()
    s.close()
    assert np.all(np.isfinite(clb)) and np.all(np.isfinite(cdb))


def test_graph_replay_equals_eager(ql, clouds):
    _say("graph vs eager")
    out = []
    for graph in (False, True):
        s = ql.Solver(limiter=1)
        s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
        s.init_freestream()
        iters, res = s.batch_run(1e-30, 40, check_every=10, graph=graph)
        out.append((s.fetch_state(), iters, res))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
    assert list(out[0][1]) == [40] * len(CASES)


def test_retirement_matches_solo(ql, clouds):
    _say("retirement")
    drops = 0.3
    s = ql.Solver(limiter=1)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    s.init_freestream()
    iters, res = s.batch_run(drops, 400, check_every=1, graph=False)
    Ub = s.fetch_state()
    s.close()
    for i, (cl, case) in enumerate(zip(clouds, CASES)):
        _, h = _solo(ql, cl, case, 400, limiter=1)
        k = int(np.argmax(h[:, 0] <= drops * h[0, 0])) + 1
        assert h[k - 1, 0] <= drops * h[0, 0]
        assert iters[i] == k, (i, iters[i], k)
        U, _ = _solo(ql, cl, case, k, limiter=1)
        np.testing.assert_array_equal(Ub[:, offs[i]:offs[i + 1]], U)
