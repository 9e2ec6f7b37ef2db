"""Edge cases through the C ABI.

Malformed uploads (empty cloud, oversized n, broken CSR, bad kinds, normals,
coordinates and split flags) and a degenerate one (an isolated point) are
rejected with a status and a message that names the point or entry, and
the solver stays usable for a valid upload afterwards.  A cloud whose last
64-point tile is partly filled matches the oracle like the full-tile
clouds: one evaluation to the evaluation tolerances, 30 iterations to
1e-11 per state component.  Out-of-range parameters are refused and leave
the solver usable.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from cloudgen import naca_ocloud
from tests._common import normwise_rel, smooth_state

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


def test_upload_rejections(ql):
    _say("upload rejections")
    c = naca_ocloud(48, 16)
    base = dict(x=c.x, y=c.y, nx=c.nx, ny=c.ny, kind=c.kind, nbr_ptr=c.nbr_ptr,
                nbr_idx=c.nbr_idx)
    s = ql.Solver()

    def expect(code, text, flag=None, **mod):
        d = {k: np.array(v, copy=True) for k, v in base.items()}
        d.update(mod)
        with pytest.raises(ql.QLError) as e:
            ql.ql_upload_cloud(s.h, d["x"], d["y"], d["nx"], d["ny"], d["kind"], d["nbr_ptr"],
                               d["nbr_idx"], flag)
        assert e.value.code == code, (text, e.value)
        assert text in str(e.value), (text, str(e.value))

    empty = np.zeros(0)
    expect(ql.QL_EINVAL, "out of range", x=empty, y=empty, nx=empty, ny=empty,
           kind=np.zeros(0, np.uint8), nbr_ptr=np.zeros(1, np.int32),
           nbr_idx=np.zeros(0, np.int32))
    kind = c.kind.copy()
    kind[5] = 3
    expect(ql.QL_EINVAL, "bad kind 3 at point 5", kind=kind)
    k = int(c.nbr_ptr[10])
    idx = c.nbr_idx.copy()
    idx[k] = 10
    expect(ql.QL_EINVAL, f"neighbour entry {k} of point 10", nbr_idx=idx)
    idx = c.nbr_idx.copy()
    idx[k] = c.n
    expect(ql.QL_EINVAL, f"neighbour entry {k} of point 10", nbr_idx=idx)
    ptr = c.nbr_ptr.copy()
    ptr[20] = ptr[19] - 1
    expect(ql.QL_EINVAL, "nbr_ptr decreases at point 19", nbr_ptr=ptr)
    ptr = c.nbr_ptr.copy()
    ptr[0] = 1
    expect(ql.QL_EINVAL, "nbr_ptr[0] must be 0", nbr_ptr=ptr)
    nx = c.nx.copy()
    nx[3] *= 1.01
    expect(ql.QL_EINVAL, "normal of point 3 is not unit", nx=nx)
    x = c.x.copy()
    x[4] = np.inf
    expect(ql.QL_EINVAL, "non-finite coordinate at point 4", x=x)
    flag = np.zeros(c.nnz, np.uint8)
    flag[7] = 0x10
    expect(ql.QL_EINVAL, "bad split flag at entry 7", flag=flag)
    # an isolated point: no stencil at all
    one = np.zeros(1)
    expect(ql.QL_ESINGULAR, "point 0", x=one, y=one, nx=one, ny=np.ones(1),
           kind=np.zeros(1, np.uint8), nbr_ptr=np.zeros(2, np.int32),
           nbr_idx=np.zeros(0, np.int32))
    # n beyond the library's limit is refused before any array is read
    buf = (C.c_double * 1)()
    ib = (C.c_int32 * 2)()
    ub = (C.c_uint8 * 1)()
    rc = ql.lib.ql_upload_cloud(s.h, C.c_int64(1 << 31), buf, buf, buf, buf, ub, ib, ib, None)
    assert rc == ql.QL_EINVAL and "out of range" in ql.lib.ql_last_error(s.h).decode()
    # still usable
    s.upload(c)
    s.init_freestream()
    hist = s.step(3)
    assert np.all(np.isfinite(hist))
    s.close()


@pytest.mark.parametrize("limiter", [0, 1])
def test_ragged_tile_parity(ql, limiter):
    """50 x 21 = 1,050 points: 16 full tiles and one of 26 points."""
    _say(f"ragged tile limiter={limiter}")
    c = naca_ocloud(50, 21)
    assert c.n % 64 != 0
    prm = dict(limiter=limiter, mach=0.85 if limiter else 0.63, alpha_deg=1.0 if limiter else 2.0)
    o = oracle.Oracle(c, oracle.params(**prm))
    o.require_valid()
    s = ql.Solver(c, **prm)
    np.testing.assert_array_equal(s.flags(), o.flag)
    U = smooth_state(c, mach=prm["mach"], alpha_deg=prm["alpha_deg"])
    s.set_state(U)
    gpu = s.evaluate()
    ora = o.evaluate(U)
    for key, tol in (("q", 1e-13), ("g", 1e-12), ("R", 5e-12), ("dt", 1e-14)):
        err = normwise_rel(gpu[key], ora[key])
        assert np.all(err <= tol), (key, err)
    if limiter:
        for key in ("qmax", "qmin"):
            assert np.all(normwise_rel(gpu[key], ora[key]) <= 1e-15), key
    s.init_freestream()
    U0 = s.fetch_state()
    s.step(30)
    U1, _ = o.run(U0, 30)
    err = normwise_rel(s.fetch_state(), U1)
    _say(f"  30 iterations: {err}")
    assert np.all(err <= 1e-11), err
    s.close()


def test_parameter_rejections(ql):
    """Out-of-range parameters are refused by ql_set_params with QL_EINVAL
    and leave the solver's parameters as they were; NULL solvers are refused
    by the progress setter."""
    _say("parameter rejections")
    c = naca_ocloud(48, 16)
    s = ql.Solver(c, precision=1)
    for bad in (dict(mixed_grad=2), dict(mixed_grad=-1), dict(mixed_switch=1.0),
                dict(mixed_switch=-1e-3), dict(precision=2), dict(grad_lds=200 * 1024),
                dict(n_inner=-1), dict(cfl=0.0), dict(outer_bc=2), dict(flux_split=3)):
        with pytest.raises(ql.QLError) as e:
            s.set_params(**bad)
        assert e.value.code == ql.QL_EINVAL, bad
    # still usable with the parameters it had
    s.init_freestream()
    h = s.step(3)
    assert np.all(np.isfinite(h))
    s.close()
    assert ql.lib.ql_set_progress(None, ql.PROGRESS_FN(), None) == ql.QL_EINVAL
