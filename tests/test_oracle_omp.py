"""The OpenMP build of the oracle (used only to time the CPU baseline on every
host core) gives the serial build's results bit for bit, and reports the
same failing point."""
import numpy as np
import pytest

import oracle
from tests._common import cloud, smooth_state


@pytest.fixture(scope="module")
def libs():
    oracle.build_omp()
    return oracle.load(), oracle.load(oracle.OMP_LIB)


def test_threads(libs):
    ser, omp = libs
    assert ser.ora_num_threads() == 1
    assert omp.ora_num_threads() >= 1


@pytest.mark.parametrize("outer_bc", [0, 1])
@pytest.mark.parametrize("limiter", [0, 1])
def test_bitwise_equal_runs(libs, limiter, outer_bc):
    ser, omp = libs
    c = cloud("jitter")
    mach, alpha = (0.85, 1.0) if limiter else (0.63, 2.0)
    prm = oracle.params(limiter=limiter, mach=mach, alpha_deg=alpha, outer_bc=outer_bc)
    U0 = smooth_state(c, mach=mach, alpha_deg=alpha)
    a = oracle.Oracle(c, prm, lib=ser)
    b = oracle.Oracle(c, prm, lib=omp)
    Ua, ha = a.run(U0, 5)
    Ub, hb = b.run(U0, 5)
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(ha, hb)
    ea, eb = a.evaluate(Ua), b.evaluate(Ua)
    for k in ea:
        np.testing.assert_array_equal(ea[k], eb[k])


def test_same_failing_point(libs):
    """Two points with a negative pressure: both builds name the smaller."""
    ser, omp = libs
    c = cloud("jitter")
    U = smooth_state(c)
    bad = [c.n - 7, 123]
    U[3, bad] = -1.0
    for lib in libs:
        o = oracle.Oracle(c, oracle.params(), lib=lib)
        with pytest.raises(oracle.OracleError) as e:
            o.evaluate(U)
        assert e.value.code == oracle.EPOSITIVITY and e.value.point == min(bad)


def test_fma_builds_bitwise_equal():
    """The OpenMP build of the FMA-contracted oracle (the noise-floor
    reference of the full-size GPU checks) gives the serial FMA build's
    results bit for bit."""
    oracle.build_omp_fma()
    ser, omp = oracle.load(oracle.FMA_LIB), oracle.load(oracle.OMP_FMA_LIB)
    c = cloud("jitter")
    prm = oracle.params(limiter=1, mach=0.85, alpha_deg=1.0)
    U0 = smooth_state(c, mach=0.85, alpha_deg=1.0)
    Ua, ha = oracle.Oracle(c, prm, lib=ser).run(U0, 5)
    Ub, hb = oracle.Oracle(c, prm, lib=omp).run(U0, 5)
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(ha, hb)
