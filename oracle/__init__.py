"""ctypes binding of the FP64 CPU oracle (oracle/qlskum_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The solver package never does.

Arrays follow the oracle's layouts: U, q, R are (4, n) component-major;
g is (8, n) with q_x in rows 0..3 and q_y in rows 4..7.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qlskum_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ESINGULAR, ENOMEM, ENONFINITE, EPOSITIVITY = 0, -1, -2, -3, -5, -6
S_PLUS, S_MINUS, N_PLUS, N_MINUS = 1, 2, 4, 8


FMA_LIB = os.path.join(_HERE, "liboracle_fma.so")


def build(cflags=("-O2", "-ffp-contract=off"), out=_LIB):
    """Compile the oracle with gcc (no FMA contraction) into a shared library."""
    # a per-process temporary: parallel test workers may build at once
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc", "-std=c99", *cflags, "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_fma():
    """The same source with FMA contraction: a second, equally valid FP64
    evaluation whose distance from the first measures the rounding noise
    floor of a problem (used to set tolerances where conditioning is poor)."""
    return build(cflags=("-O2", "-mfma", "-ffp-contract=fast"), out=FMA_LIB)


OMP_LIB = os.path.join(_HERE, "liboracle_omp.so")


def build_omp():
    """The same source with OpenMP: the loops over points run on every host
    core (OMP_NUM_THREADS), with results bit for bit those of the serial
    build.  Used only to time the CPU baseline."""
    return build(cflags=("-O2", "-ffp-contract=off", "-fopenmp"), out=OMP_LIB)


OMP_FMA_LIB = os.path.join(_HERE, "liboracle_omp_fma.so")


def build_omp_fma():
    """The FMA-contracted build with OpenMP: the noise-floor reference of
    build_fma() for runs on whole large clouds."""
    return build(cflags=("-O2", "-mfma", "-ffp-contract=fast", "-fopenmp"), out=OMP_FMA_LIB)


class OracleError(RuntimeError):
    def __init__(self, code, point):
        super().__init__(f"oracle status {code} at point {point}")
        self.code, self.point = code, point


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mach", C.c_double), ("alpha_deg", C.c_double),
                ("cfl", C.c_double), ("n_inner", C.c_int32), ("limiter", C.c_int32),
                ("venkat_k", C.c_double), ("order", C.c_int32), ("outer_bc", C.c_int32)]


class _Cloud(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("nx", C.c_void_p),
                ("ny", C.c_void_p), ("kind", C.c_void_p), ("ptr", C.c_void_p),
                ("idx", C.c_void_p), ("flag", C.c_void_p)]


_lib_cache = {}

# A test of the pins' sensitivity loads a deliberately altered build of the
# oracle from this path instead (it is never rebuilt from the source here).
_OVERRIDE = os.environ.get("QL_ORACLE_LIB")


def load(path=_LIB):
    if path == _LIB and _OVERRIDE:
        path = _OVERRIDE
    if path in _lib_cache:
        return _lib_cache[path]
    if path == _OVERRIDE:
        pass
    elif not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        if path == _LIB:
            build()
        elif path == FMA_LIB:
            build_fma()
        elif path == OMP_LIB:
            build_omp()
        elif path == OMP_FMA_LIB:
            build_omp_fma()
        else:
            raise FileNotFoundError(path)
    lib = C.CDLL(path)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    P = C.POINTER
    lib.ora_num_threads.argtypes = []
    lib.ora_num_threads.restype = C.c_int
    lib.ora_classify.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, P(i64)]
    lib.ora_q_variables.argtypes = [i64, vp, d, vp, P(i64)]
    lib.ora_q_derivatives.argtypes = [P(_Cloud), i32, vp, vp, vp, vp]
    lib.ora_flux_residual.argtypes = [P(_Cloud), P(_Params), vp, vp, vp, vp, vp, P(i64)]
    lib.ora_timestep.argtypes = [P(_Cloud), P(_Params), vp, vp]
    lib.ora_state_update.argtypes = [P(_Cloud), P(_Params), i32, vp, vp, vp, vp]
    lib.ora_rk_stage.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    lib.ora_residue.argtypes = [P(_Cloud), P(_Params), vp, vp]
    lib.ora_evaluate.argtypes = [P(_Cloud), P(_Params), vp, vp, vp, vp, vp, vp, vp, P(i64)]
    lib.ora_run.argtypes = [P(_Cloud), P(_Params), vp, i32, vp, P(i64)]
    lib.ora_forces.argtypes = [P(_Cloud), P(_Params), vp, P(d), P(d)]
    lib.ora_freestream.argtypes = [i64, vp, vp, vp, P(_Params), C.c_int, vp]
    lib.ora_split_flux.argtypes = [vp, d, d, C.c_int, d, vp]
    lib.ora_venkat.argtypes = [d, d, d, d, d]
    lib.ora_venkat.restype = d
    lib.ora_venkat_eps2.argtypes = [d, d, d]
    lib.ora_venkat_eps2.restype = d
    lib.ora_modified_q.argtypes = [P(_Cloud), P(_Params), vp, vp, vp, vp, i64, i64, vp, vp]
    for f in ("ora_u_to_prim", "ora_prim_to_u", "ora_prim_to_q", "ora_q_to_prim"):
        getattr(lib, f).argtypes = [vp, d, vp]
    _lib_cache[path] = lib
    return lib


def _p(a):
    return a.ctypes.data if a is not None else None


def params(gamma=1.4, mach=0.63, alpha_deg=2.0, cfl=0.2, n_inner=3, limiter=0, venkat_k=5.0,
           order=2, outer_bc=0):
    """order 2: modified q of eq. (28) (second order); 1: first-order LSKUM,
    the split fluxes of q itself.  outer_bc 0: outer points held at the
    freestream; 1: kinetic outer condition."""
    return dict(gamma=gamma, mach=mach, alpha_deg=alpha_deg, cfl=cfl, n_inner=n_inner,
                limiter=limiter, venkat_k=venkat_k, order=order, outer_bc=outer_bc)


class Oracle:
    """One cloud bound to the oracle; arrays are kept alive here."""

    def __init__(self, cloud, prm=None, lib=None):
        self.lib = lib or load()
        self.cloud = cloud
        self.n = cloud.n
        self.x = np.ascontiguousarray(cloud.x, np.float64)
        self.y = np.ascontiguousarray(cloud.y, np.float64)
        self.nx = np.ascontiguousarray(cloud.nx, np.float64)
        self.ny = np.ascontiguousarray(cloud.ny, np.float64)
        self.kind = np.ascontiguousarray(cloud.kind, np.uint8)
        self.ptr = np.ascontiguousarray(cloud.nbr_ptr, np.int32)
        self.idx = np.ascontiguousarray(cloud.nbr_idx, np.int32)
        self.flag = np.zeros(self.idx.shape[0], np.uint8)
        bad = C.c_int64(-1)
        st = self.lib.ora_classify(self.n, _p(self.x), _p(self.y), _p(self.nx), _p(self.ny),
                                   _p(self.kind), _p(self.ptr), _p(self.idx), _p(self.flag),
                                   C.byref(bad))
        self.classify_status, self.classify_point = st, bad.value
        self._c = _Cloud(self.n, _p(self.x), _p(self.y), _p(self.nx), _p(self.ny),
                         _p(self.kind), _p(self.ptr), _p(self.idx), _p(self.flag))
        self.set_params(**(prm or params()))

    def require_valid(self):
        if self.classify_status != OK:
            raise OracleError(self.classify_status, self.classify_point)

    def set_params(self, **kw):
        base = params()
        base.update(getattr(self, "prm", {}))
        base.update(kw)
        self.prm = base
        self._prm = _Params(**base)

    def freestream(self, project_wall=True):
        U = np.empty((4, self.n))
        self.lib.ora_freestream(self.n, _p(self.nx), _p(self.ny), _p(self.kind),
                                C.byref(self._prm), int(project_wall), _p(U))
        return U

    def evaluate(self, U):
        """One evaluation of the stage operator at U."""
        self.require_valid()
        U = np.ascontiguousarray(U, np.float64)
        n = self.n
        q, g = np.empty((4, n)), np.empty((8, n))
        qmax, qmin, R, dt = np.empty((4, n)), np.empty((4, n)), np.empty((4, n)), np.empty(n)
        bad = C.c_int64(-1)
        st = self.lib.ora_evaluate(C.byref(self._c), C.byref(self._prm), _p(U), _p(q), _p(g),
                                   _p(qmax), _p(qmin), _p(R), _p(dt), C.byref(bad))
        if st:
            raise OracleError(st, bad.value)
        return dict(q=q, g=g, qmax=qmax, qmin=qmin, R=R, dt=dt)

    def q_derivatives(self, q, n_inner):
        q = np.ascontiguousarray(q, np.float64)
        n = self.n
        g, qmax, qmin = np.empty((8, n)), np.empty((4, n)), np.empty((4, n))
        self.lib.ora_q_derivatives(C.byref(self._c), int(n_inner), _p(q), _p(g), _p(qmax),
                                   _p(qmin))
        return g, qmax, qmin

    def timestep(self, U):
        """Local time step of Algorithm 1's timestep() at U, (n,)."""
        U = np.ascontiguousarray(U, np.float64)
        dt = np.empty(self.n)
        self.lib.ora_timestep(C.byref(self._c), C.byref(self._prm), _p(U), _p(dt))
        return dt

    def residue(self, R):
        """residue() of a (4, n) residual array: RMS over interior and wall."""
        R = np.ascontiguousarray(R, np.float64)
        out = np.empty(4)
        self.lib.ora_residue(C.byref(self._c), C.byref(self._prm), _p(R), _p(out))
        return out

    def modified_q(self, q, g, qmax, qmin, p, k):
        """The two modified states (q~_i, q~_0) of eq. (28) for neighbour
        entry k of point p."""
        q, g, qmax, qmin = (np.ascontiguousarray(a, np.float64) for a in (q, g, qmax, qmin))
        qti, qt0 = np.empty(4), np.empty(4)
        self.lib.ora_modified_q(C.byref(self._c), C.byref(self._prm), _p(q), _p(g), _p(qmax),
                                _p(qmin), int(p), int(k), _p(qti), _p(qt0))
        return qti, qt0

    def run(self, U, n_iter):
        """n_iter iterations from U; returns (U_new, residual history (n_iter, 4))."""
        self.require_valid()
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        hist = np.zeros((max(n_iter, 1), 4))
        bad = C.c_int64(-1)
        st = self.lib.ora_run(C.byref(self._c), C.byref(self._prm), _p(U), int(n_iter),
                              _p(hist), C.byref(bad))
        if st:
            raise OracleError(st, bad.value)
        return U, hist[:n_iter]

    def forces(self, U):
        U = np.ascontiguousarray(U, np.float64)
        cl, cd = C.c_double(), C.c_double()
        st = self.lib.ora_forces(C.byref(self._c), C.byref(self._prm), _p(U), C.byref(cl),
                                 C.byref(cd))
        if st:
            raise OracleError(st, -1)
        return cl.value, cd.value


def _vec4(fn, v, gamma):
    lib = load()
    a = np.ascontiguousarray(v, np.float64)
    out = np.empty(4)
    getattr(lib, fn)(_p(a), gamma, _p(out))
    return out


def u_to_prim(U, gamma=1.4):
    return _vec4("ora_u_to_prim", U, gamma)


def prim_to_u(prim, gamma=1.4):
    return _vec4("ora_prim_to_u", prim, gamma)


def prim_to_q(prim, gamma=1.4):
    return _vec4("ora_prim_to_q", prim, gamma)


def q_to_prim(q, gamma=1.4):
    return _vec4("ora_q_to_prim", q, gamma)


def split_flux(prim, e, sign, gamma=1.4):
    lib = load()
    a = np.ascontiguousarray(prim, np.float64)
    G = np.empty(4)
    lib.ora_split_flux(_p(a), float(e[0]), float(e[1]), int(sign), gamma, _p(G))
    return G


def venkat(delta, q, qmax, qmin, eps2):
    """The limiter value phi for one increment (see ora_venkat)."""
    return load().ora_venkat(float(delta), float(q), float(qmax), float(qmin), float(eps2))


def venkat_eps2(K, dx, dy):
    return load().ora_venkat_eps2(float(K), float(dx), float(dy))


def rk_stage(rk, un, u, r, dt):
    lib = load()
    un, u, r, dt = (np.ascontiguousarray(a, np.float64) for a in (un, u, r, dt))
    out = np.empty_like(u)
    lib.ora_rk_stage(int(rk), u.shape[0], _p(un), _p(u), _p(r), _p(dt), _p(out))
    return out
