"""The sampled full-size checks evaluate the oracle on dependency sub-clouds
(tests/_common.py: dependency_subcloud).  Here, on clouds the oracle solves
whole in well under a second, the sub-cloud values at the sampled points
must equal the whole-cloud values bit for bit, and one ring fewer must not
(the flux residual reaches n_inner + 2 neighbour hops: the final
q-derivatives of the neighbours, eq. (28) and the inner iterations of
eq. (29))."""
import numpy as np
import pytest

import oracle
from tests._common import cloud, dependency_subcloud, sample_points, smooth_state


@pytest.mark.parametrize("name,limiter,order", [("jitter", 1, 2), ("c1", 0, 2), ("jitter", 0, 1)])
def test_dependency_subcloud_matches_whole_cloud(oracle_lib, name, limiter, order):
    c = cloud(name)
    flow = dict(mach=0.85, alpha_deg=1.0) if limiter else dict(mach=0.63, alpha_deg=2.0)
    prm = oracle.params(limiter=limiter, order=order, **flow)
    U = smooth_state(c, **flow)
    full = oracle.Oracle(c, prm).evaluate(U)
    centres = sample_points(c, 48, seed=11)
    depth = prm["n_inner"] + 2 if order == 2 else 1
    sub, members, where = dependency_subcloud(c, centres, depth)
    assert sub.n < c.n
    part = oracle.Oracle(sub, prm).evaluate(U[:, members])
    # first order: the residual reaches one hop; the q-derivatives (still
    # computed) are then not compared
    keys = ("q", "g", "qmax", "qmin", "R", "dt") if order == 2 else ("q", "qmax", "qmin", "R", "dt")
    for key in keys:
        np.testing.assert_array_equal(np.atleast_2d(part[key])[:, where],
                                      np.atleast_2d(full[key])[:, centres], err_msg=key)
    # one ring fewer changes the residual somewhere
    sub2, members2, where2 = dependency_subcloud(c, centres, depth - 1)
    if depth > 1:
        part2 = oracle.Oracle(sub2, prm).evaluate(U[:, members2])
        assert np.any(part2["R"][:, where2] != full["R"][:, centres])


def test_dependency_subcloud_one_iteration(oracle_lib):
    """A whole pseudo-time iteration (four stages, each reaching n_inner + 2
    hops) on sub-clouds of depth 4 (n_inner + 2) + 1 gives the whole-cloud
    state at the sampled points bit for bit (400 x 300 jittered cloud,
    limiter on)."""
    from cloudgen import naca_ocloud
    c = naca_ocloud(400, 300, jitter=0.1, seed=5)
    flow = dict(mach=0.85, alpha_deg=1.0)
    prm = oracle.params(limiter=1, **flow)
    U = smooth_state(c, **flow)
    full, _ = oracle.Oracle(c, prm).run(U, 1)
    centres = sample_points(c, 12, seed=13)
    depth = 4 * (prm["n_inner"] + 2) + 1
    sub, members, where = dependency_subcloud(c, centres, depth)
    assert sub.n < c.n
    part, _ = oracle.Oracle(sub, prm).run(U[:, members], 1)
    np.testing.assert_array_equal(part[:, where], full[:, centres])
