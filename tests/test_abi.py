"""The C-ABI library loads and exports every entry point the public header
declares; argument checks that need no GPU."""
import ctypes as C
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qlskum.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ql_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2108_07031_amd import qlskum
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(qlskum.lib, name), name
    assert set(names) == set(qlskum.EXPORTS)


def test_host_side_checks_without_gpu():
    from paper_2108_07031_amd import qlskum as q
    p = q.ql_default_params()
    assert (p.gamma, p.mach, p.alpha_deg, p.cfl, p.n_inner, p.limiter) == (1.4, 0.63, 2.0, 0.2, 3, 0)
    assert (p.precision, p.reorder, p.flux_lds, p.grad_lds, p.order, p.flux_split) == \
        (0, 1, 0, 0, 2, 0)
    h = C.c_void_p()
    assert q.lib.ql_create(None, 0, None) == q.QL_EINVAL
    rc = q.lib.ql_create(C.byref(h), -1, None)
    assert rc == q.QL_EDEVICE and not h.value
    assert q.lib.ql_destroy(None) == q.QL_OK
    out = (C.c_double * 4)()
    assert q.lib.ql_residual_norm(None, out) == q.QL_EINVAL


def test_params_struct_layout():
    from paper_2108_07031_amd import qlskum as q
    # doubles and int32s as in the header: 4 d, 2 i32, 1 d, 6 i32
    assert C.sizeof(q.ql_params) == 4 * 8 + 2 * 4 + 8 + 6 * 4
    assert q.ql_params.order.offset == 4 * 8 + 2 * 4 + 8 + 4 * 4
    assert q.ql_params.flux_lds.offset == 4 * 8 + 2 * 4 + 8 + 2 * 4
    assert q.ql_params.grad_lds.offset == 4 * 8 + 2 * 4 + 8 + 3 * 4
