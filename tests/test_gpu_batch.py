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


@pytest.mark.parametrize("check_every,graph", [(1, False), (1, True), (50, False), (50, True)])
def test_retirement_matches_solo(ql, clouds, check_every, graph):
    """Retirement happens on the device after every iteration, so a case
    that reaches the drop in the middle of a check window keeps exactly the
    state of a solo run of that many iterations, and reports the norm of
    that iteration.  After a window with retirements the tiled sweeps run
    over the live tiles only (with check_every 1 and graph replay the
    iteration is re-captured after every retirement); the cases still
    running are unaffected bit for bit."""
    _say(f"retirement check_every={check_every} graph={graph}")
    drops = 0.3
    s = ql.Solver(limiter=1)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    s.init_freestream()
    iters, res = s.batch_run(drops, 400, check_every=check_every, graph=graph)
    Ub = s.fetch_state()
    assert list(s.batch_status()) == [ql.QL_OK] * len(CASES)
    s.close()
    ks = []
    for i, (cl, case) in enumerate(zip(clouds, CASES)):
        _, h = _solo(ql, cl, case, 400, limiter=1)
        k = int(np.argmax(h[:, 0] <= drops * h[0, 0])) + 1
        assert h[k - 1, 0] <= drops * h[0, 0]
        assert iters[i] == k, (i, iters[i], k)
        np.testing.assert_array_equal(res[i], h[k - 1])
        U, _ = _solo(ql, cl, case, k, limiter=1)
        np.testing.assert_array_equal(Ub[:, offs[i]:offs[i + 1]], U)
        ks.append(k)
    _say(f"  crossing iterations {ks}")
    # the crossings fall inside windows, not on their ends
    assert any(k % 50 != 0 for k in ks)


def test_batched_cases_match_oracle(ql, clouds):
    """Each case of the batch after 30 FP64 iterations from its freestream
    equals the oracle's run of that case's cloud at its own Mach number and
    incidence: 1e-11 normwise per state component (the FP64 parity bound)
    and 1e-10 relative on every residual norm of the history."""
    import oracle
    from tests._common import normwise_rel
    _say("batched FP64 vs oracle")
    s = ql.Solver(limiter=1)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    s.init_freestream()
    hb = s.step(30)
    Ub = s.fetch_state()
    s.close()
    for i, (cl, case) in enumerate(zip(clouds, CASES)):
        o = oracle.Oracle(cl, oracle.params(limiter=1, mach=case["mach"],
                                            alpha_deg=case["alpha"]))
        Uo, ho = o.run(o.freestream(), 30)
        err = normwise_rel(Ub[:, offs[i]:offs[i + 1]], Uo)
        herr = np.abs(hb[:, i] - ho).max() / np.abs(ho).max()
        _say(f"  case {i}: state {err.max():.2e}, history {herr:.2e}")
        assert np.all(err <= 1e-11), (i, err)
        assert herr <= 1e-10, (i, herr)


def test_batched_mixed_evaluate_matches_oracle(ql, clouds):
    """Mixed precision on the batch: one evaluation of every case at a
    smooth state lies within the mixed evaluation bound (2e-3 normwise per
    component) of the oracle's FP64 evaluation of that case alone."""
    import oracle
    from tests._common import normwise_rel, smooth_state
    _say("batched mixed evaluate vs oracle")
    s = ql.Solver(limiter=1, precision=1)
    offs = s.upload_batch(clouds, [c["mach"] for c in CASES], [c["alpha"] for c in CASES])
    Us = [smooth_state(cl, mach=case["mach"], alpha_deg=case["alpha"])
          for cl, case in zip(clouds, CASES)]
    s.set_state(np.concatenate(Us, axis=1))
    R = s.evaluate()["R"]
    s.close()
    for i, (cl, case) in enumerate(zip(clouds, CASES)):
        o = oracle.Oracle(cl, oracle.params(limiter=1, mach=case["mach"],
                                            alpha_deg=case["alpha"]))
        err = normwise_rel(R[:, offs[i]:offs[i + 1]], o.evaluate(Us[i])["R"])
        _say(f"  case {i}: R {err}")
        assert np.all(err <= 2e-3), (i, err)


def _bad_point_state(cl_list, offs, U0, cases):
    """U0 with one interior point's pressure set to 1e-6 in each listed case
    (the reconstruction next to it then gives q~4 >= 0)."""
    bad = U0.copy()
    for c in cases:
        cl = cl_list[c]
        lp = (cl.meta["nr"] // 2) * cl.meta["ns"] + 7
        assert cl.kind[lp] == 0
        p0 = int(offs[c]) + lp
        rho, m1, m2 = bad[0, p0], bad[1, p0], bad[2, p0]
        bad[3, p0] = 1e-6 / 0.4 + 0.5 * (m1 * m1 + m2 * m2) / rho
    return bad


@pytest.mark.parametrize("n_iter,check_every", [(200, 50), (50, 50)])
def test_two_failed_cases_in_one_window(ql, clouds, n_iter, check_every):
    """Cases 1 and 3 of four fail in the same check window (with n_iter =
    check_every it is also the last window): both retire with a failure
    status, and cases 0 and 2 run on bit for bit as in the same batch
    without the failures."""
    _say(f"two failed cases n_iter={n_iter}")
    cl = [clouds[0], clouds[1], clouds[0], clouds[1]]
    mach, alpha = [0.63, 0.5, 0.4, 0.55], [2.0, -1.5, 0.0, 1.0]

    def batch(U, n):
        s = ql.Solver(limiter=0)
        offs = s.upload_batch(cl, mach, alpha)
        if U is None:
            s.init_freestream()
        else:
            s.set_state(U)
        iters, _ = s.batch_run(1e-300, n, check_every=check_every, graph=True)
        return s, offs, iters

    s, offs, _ = batch(None, 0)
    U0 = s.fetch_state()
    s.close()
    s, _, _ = batch(U0, n_iter)
    Uref = s.fetch_state()
    assert list(s.batch_status()) == [ql.QL_OK] * 4
    s.close()
    s, _, iters = batch(_bad_point_state(cl, offs, U0, (1, 3)), n_iter)
    status = s.batch_status()
    _say(f"  status {status}, iterations {iters}")
    for c in (1, 3):
        assert status[c] in (ql.QL_EPOSITIVITY, ql.QL_ENONFINITE), (c, status)
        assert 1 <= iters[c] < n_iter
    U = s.fetch_state()
    s.close()
    for c in (0, 2):
        assert status[c] == ql.QL_OK and iters[c] == n_iter
        lo, hi = int(offs[c]), int(offs[c + 1])
        np.testing.assert_array_equal(U[:, lo:hi], Uref[:, lo:hi])


def test_step_without_history_defers_its_status(ql, clouds):
    """ql_step without a history returns once its work is enqueued; the next
    call collects the outcome: the last norms equal those of a run with a
    history, and a failure during the iterations is returned by the call
    that collects it."""
    _say("step without history")
    cl, case = clouds[0], CASES[0]
    s = ql.Solver(cl, mach=case["mach"], alpha_deg=case["alpha"], limiter=1)
    s.init_freestream()
    assert s.step(12, want_history=False) is None
    r = s.residual_norm()
    U = s.fetch_state()
    s.close()
    Us, h = _solo(ql, cl, case, 12, limiter=1)
    np.testing.assert_array_equal(r, h[-1])
    np.testing.assert_array_equal(U, Us)
    s = ql.Solver(cl, mach=case["mach"], alpha_deg=case["alpha"], limiter=0)
    s.init_freestream()
    offs = np.array([0, cl.n])
    s.set_state(_bad_point_state([cl], offs, s.fetch_state(), (0,)))
    assert s.step(3, want_history=False) is None
    with pytest.raises(ql.QLError) as ei:
        s.fetch_state()
    assert ei.value.code in (ql.QL_EPOSITIVITY, ql.QL_ENONFINITE)
    s.close()


@pytest.mark.parametrize("graph", [True, False])
def test_failed_case_retires_alone(ql, clouds, graph):
    """Three cases without the limiter at conditions that run stably (M 0.63,
    0.5 and 0.4); in the middle one a point's pressure is set to 1e-6, so
    the reconstruction next to it gives q~4 >= 0 and the case fails.  It is
    retired with its status within the first check window while the other
    two run on; their states equal those of the same batch without the
    failure bit for bit, and the solver runs on once every case has a valid
    state again."""
    _say(f"failed case graph={graph}")
    prm = dict(limiter=0)
    cl = [clouds[0], clouds[1], clouds[0]]
    mach, alpha = [0.63, 0.5, 0.4], [2.0, -1.5, 0.0]

    def batch(U=None, n=200):
        s = ql.Solver(**prm)
        offs = s.upload_batch(cl, mach, alpha)
        if U is None:
            s.init_freestream()
        else:
            s.set_state(U)
        iters, _ = s.batch_run(1e-300, n, check_every=50, graph=graph)
        return s, offs, iters

    ref, offs, _ = batch()
    assert list(ref.batch_status()) == [ql.QL_OK] * 3
    ref.close()
    ref, _, _ = batch(n=0)
    U0 = ref.fetch_state()
    ref.close()
    ref, _, _ = batch(U0)
    Uref = ref.fetch_state()
    ref.close()
    bad = U0.copy()
    c1 = cl[1]
    lp = (c1.meta["nr"] // 2) * c1.meta["ns"] + 7  # an interior point of case 1
    assert c1.kind[lp] == 0
    p0 = int(offs[1]) + lp
    rho, m1, m2 = bad[0, p0], bad[1, p0], bad[2, p0]
    bad[3, p0] = 1e-6 / 0.4 + 0.5 * (m1 * m1 + m2 * m2) / rho
    s, _, iters = batch(bad)
    status = s.batch_status()
    _say(f"  status {status}, iterations {iters}")
    assert status[0] == ql.QL_OK and status[2] == ql.QL_OK
    assert status[1] in (ql.QL_EPOSITIVITY, ql.QL_ENONFINITE)
    assert iters[0] == 200 and iters[2] == 200 and iters[1] <= 50
    U = s.fetch_state()
    for k in (0, 2):
        lo, hi = int(offs[k]), int(offs[k + 1])
        np.testing.assert_array_equal(U[:, lo:hi], Uref[:, lo:hi])
    # every case valid again: the solver runs on, all statuses clear
    s.set_state(U0)
    s.batch_run(1e-300, 20, check_every=10, graph=graph)
    assert list(s.batch_status()) == [ql.QL_OK] * 3
    s.close()


def test_progress_callback(ql):
    """ql_set_progress: one call per check window with the iterations done so
    far and the cases still active, the last at the run's end."""
    _say("progress callback")
    clouds = [naca_ocloud(48, 16), naca_ocloud(40, 16, tau=0.1)]
    s = ql.Solver(limiter=0)
    s.upload_batch(clouds, [0.63, 0.5], [2.0, 1.0])
    s.init_freestream()
    calls = []
    s.set_progress(lambda it, active: calls.append((it, active)))
    iters, _ = s.batch_run(1e-300, 250, check_every=100)
    s.set_progress(None)
    s.batch_run(1e-300, 10, check_every=5)
    s.close()
    assert calls == [(100, 2), (200, 2), (250, 2)], calls
    assert list(iters) == [250, 250]
