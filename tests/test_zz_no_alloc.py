"""ql_step_static: the step entry point for callers that cannot allocate
device memory.  It runs the kernels of ql_step with the residual history in
the library's fixed per-GPU array, so its states and histories equal
ql_step's bit for bit.  Two calls in a row on one GPU, the second on a
smaller cloud with fewer iterations, check that the array's leftover rows
from the first call never reach the second's results."""
import numpy as np
import pytest

from tests._common import cloud

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ql():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2108_07031_amd import qlskum
    return qlskum


def _say(msg):
    print(msg, flush=True)


def _pair(ql, c, n_iter, **prm):
    """(history, state) of ql_step and of ql_step_static from the same start"""
    out = []
    for static in (False, True):
        s = ql.Solver(c, **prm)
        s.init_freestream()
        h = s.step_static(n_iter) if static else s.step(n_iter)
        out.append((h, s.fetch_state(), s.residual_norm()))
        s.close()
    return out


def test_static_step_equals_step(ql):
    big, small = cloud("c1"), cloud("small")
    _say(f"static step: {big.n} points x 40 iterations, then {small.n} points x 15")
    (h0, U0, r0), (h1, U1, r1) = _pair(ql, big, 40, limiter=1)
    assert h1.shape == (40, 4)
    np.testing.assert_array_equal(h1, h0)
    np.testing.assert_array_equal(U1, U0)
    np.testing.assert_array_equal(r1, r0)
    (h0, U0, r0), (h1, U1, r1) = _pair(ql, small, 15, limiter=0, mach=0.5, alpha_deg=-1.0)
    assert h1.shape == (15, 4)
    np.testing.assert_array_equal(h1, h0)
    np.testing.assert_array_equal(U1, U0)
    np.testing.assert_array_equal(r1, r0)


def test_static_step_without_history(ql):
    c = cloud("small")
    _say("static step without history")
    s = ql.Solver(c, limiter=1)
    s.init_freestream()
    h = s.step(12)
    U = s.fetch_state()
    s.close()
    s = ql.Solver(c, limiter=1)
    s.init_freestream()
    assert s.step_static(12, want_history=False) is None
    np.testing.assert_array_equal(s.residual_norm(), h[-1])
    np.testing.assert_array_equal(s.fetch_state(), U)
    s.close()


def test_static_step_rejects_too_many_rows(ql):
    c = cloud("small")
    s = ql.Solver(c)
    s.init_freestream()
    with pytest.raises(ql.QLError) as ei:
        s.step_static(65536 // 4 + 1)
    assert ei.value.code == ql.QL_EINVAL
    s.close()
