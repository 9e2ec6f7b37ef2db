"""Thin ctypes binding of libqlskum.so (include/qlskum.h).

Every function keeps the C name and only marshals arguments: numpy arrays
for host memory, torch CUDA tensors (or raw integer device pointers) for
device memory, torch's current stream for ordering.  All computation runs
in the library's HIP kernels; there is no fallback: if the library is not
built, importing this module raises.
"""
import ctypes as C
import os

import numpy as np

try:  # torch first: the process then uses torch's HIP runtime for both
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is only plumbing
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqlskum.so")

QL_OK, QL_EINVAL, QL_ESINGULAR, QL_ENOMEM, QL_EDEVICE = 0, -1, -2, -3, -4
QL_ENONFINITE, QL_EPOSITIVITY, QL_EDIVERGED, QL_ESTATE = -5, -6, -7, -8
QL_KIND_INTERIOR, QL_KIND_WALL, QL_KIND_OUTER = 0, 1, 2
QL_SPLIT_S_PLUS, QL_SPLIT_S_MINUS, QL_SPLIT_N_PLUS, QL_SPLIT_N_MINUS = 1, 2, 4, 8

# every entry point the public header declares
EXPORTS = ("ql_default_params", "ql_create", "ql_destroy", "ql_upload_cloud", "ql_set_params",
           "ql_init_freestream", "ql_set_state", "ql_step", "ql_step_static",
           "ql_residual_norm",
           "ql_fetch_state", "ql_forces", "ql_last_error", "ql_evaluate", "ql_debug_fetch",
           "ql_debug_flags", "ql_cloud_size", "ql_set_timing", "ql_kernel_time",
           "ql_batch_upload", "ql_batch_info", "ql_batch_run", "ql_batch_status",
           "ql_batch_switched", "ql_set_progress",
           "ql_batch_forces",
           "ql_flux_tiles", "ql_mlp_create", "ql_mlp_destroy", "ql_mlp_last_error",
           "ql_mlp_num_params", "ql_mlp_set_weights", "ql_mlp_get_weights", "ql_mlp_forward",
           "ql_mlp_gradient", "ql_mlp_train_step", "ql_mlp_sync", "ql_wall_distance",
           "ql_warm_start", "ql_autotune")


class ql_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mach", C.c_double), ("alpha_deg", C.c_double),
                ("cfl", C.c_double), ("n_inner", C.c_int32), ("limiter", C.c_int32),
                ("venkat_k", C.c_double), ("precision", C.c_int32), ("reorder", C.c_int32),
                ("flux_lds", C.c_int32), ("grad_lds", C.c_int32), ("order", C.c_int32),
                ("flux_split", C.c_int32), ("outer_bc", C.c_int32), ("mixed_grad", C.c_int32),
                ("mixed_switch", C.c_double)]


class QLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qlskum error {code}: {msg}")
        self.code = code


# void (*)(void *user, int32_t iterations, int32_t active)
PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2108_07031_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.ql_default_params.argtypes = [P(ql_params)]
    lib.ql_default_params.restype = None
    lib.ql_create.argtypes = [P(vp), i32, vp]
    lib.ql_destroy.argtypes = [vp]
    lib.ql_upload_cloud.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ql_set_params.argtypes = [vp, P(ql_params)]
    lib.ql_init_freestream.argtypes = [vp]
    lib.ql_set_state.argtypes = [vp, vp, i32, i32]
    lib.ql_step.argtypes = [vp, i32, vp]
    lib.ql_step_static.argtypes = [vp, i32, vp]
    lib.ql_residual_norm.argtypes = [vp, vp]
    lib.ql_fetch_state.argtypes = [vp, vp, i32]
    lib.ql_forces.argtypes = [vp, P(d), P(d)]
    lib.ql_last_error.argtypes = [vp]
    lib.ql_last_error.restype = C.c_char_p
    lib.ql_evaluate.argtypes = [vp]
    lib.ql_debug_fetch.argtypes = [vp, i32, vp]
    lib.ql_debug_flags.argtypes = [vp, vp]
    lib.ql_cloud_size.argtypes = [vp, P(i64), P(i64)]
    lib.ql_set_timing.argtypes = [vp, i32]
    lib.ql_kernel_time.argtypes = [vp, i32, P(d), P(i64)]
    lib.ql_batch_upload.argtypes = [vp, i32, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.ql_batch_info.argtypes = [vp, P(i32)]
    lib.ql_batch_run.argtypes = [vp, d, i32, i32, i32, vp, vp, vp]
    lib.ql_batch_forces.argtypes = [vp, vp, vp]
    lib.ql_flux_tiles.argtypes = [vp, P(i32), vp]
    lib.ql_mlp_create.argtypes = [P(vp), i32, vp, vp, i32, i64]
    lib.ql_mlp_destroy.argtypes = [vp]
    lib.ql_mlp_last_error.argtypes = [vp]
    lib.ql_mlp_last_error.restype = C.c_char_p
    lib.ql_mlp_num_params.argtypes = [vp, P(i64)]
    lib.ql_mlp_set_weights.argtypes = [vp, vp]
    lib.ql_mlp_get_weights.argtypes = [vp, vp]
    lib.ql_mlp_forward.argtypes = [vp, vp, vp, i64]
    lib.ql_mlp_gradient.argtypes = [vp, vp, vp, i64, vp, P(d)]
    lib.ql_mlp_train_step.argtypes = [vp, vp, vp, i64, C.c_float, P(d)]
    lib.ql_mlp_sync.argtypes = [vp]
    lib.ql_wall_distance.argtypes = [vp, vp]
    lib.ql_warm_start.argtypes = [vp, vp, vp, vp, d, vp, vp, vp]
    lib.ql_autotune.argtypes = [vp, C.c_char_p, vp]
    lib.ql_batch_status.argtypes = [vp, vp]
    lib.ql_batch_switched.argtypes = [vp, vp]
    lib.ql_set_progress.argtypes = [vp, PROGRESS_FN, vp]
    for name in EXPORTS:
        if name not in ("ql_default_params", "ql_last_error", "ql_mlp_last_error"):
            getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


def _check(s, rc):
    if rc != QL_OK:
        msg = lib.ql_last_error(s).decode() if s else ""
        raise QLError(rc, msg)
    return rc


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _dev_ptr(t):
    """Device pointer of a torch CUDA tensor (contiguous) or an int."""
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return t.data_ptr()


def ql_default_params():
    p = ql_params()
    lib.ql_default_params(C.byref(p))
    return p


def ql_create(device=0, stream=None):
    """stream: hipStream_t as int, a torch stream, or None for torch's
    current stream on `device` (the library creates its own if torch has
    no GPU)."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
    elif not isinstance(stream, int):
        stream = stream.cuda_stream
    h = C.c_void_p()
    rc = lib.ql_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
    if rc != QL_OK:
        raise QLError(rc, "ql_create failed")
    return h


def ql_destroy(s):
    return lib.ql_destroy(s)


def ql_upload_cloud(s, x, y, nx, ny, kind, nbr_ptr, nbr_idx, nbr_flag=None):
    keep = [_host(x, np.float64), _host(y, np.float64), _host(nx, np.float64),
            _host(ny, np.float64), _host(kind, np.uint8), _host(nbr_ptr, np.int32),
            _host(nbr_idx, np.int32)]
    fl = _host(nbr_flag, np.uint8) if nbr_flag is not None else (None, None)
    n = keep[0][0].shape[0]
    return _check(s, lib.ql_upload_cloud(s, n, *(k[1] for k in keep), fl[1]))


def ql_set_params(s, p):
    return _check(s, lib.ql_set_params(s, C.byref(p)))


def ql_init_freestream(s):
    return _check(s, lib.ql_init_freestream(s))


def ql_set_state(s, U, project_wall=False):
    """U: numpy (4, n) on the host, or a torch CUDA tensor (4, n) on the
    solver's device."""
    if isinstance(U, np.ndarray):
        a, ptr = _host(U, np.float64)
        return _check(s, lib.ql_set_state(s, ptr, 0, int(bool(project_wall))))
    return _check(s, lib.ql_set_state(s, _dev_ptr(U), 1, int(bool(project_wall))))


def ql_batch_info(s):
    nc = C.c_int32()
    _check(s, lib.ql_batch_info(s, C.byref(nc)))
    return nc.value


def ql_step(s, n_iter, want_history=True):
    """Returns the residual history, (n_iter, 4) for one case or
    (n_iter, ncase, 4) for a batched cloud (or None)."""
    nc = ql_batch_info(s)
    hist = np.zeros((max(n_iter, 1), nc, 4)) if want_history else None
    _check(s, lib.ql_step(s, int(n_iter), hist.ctypes.data if want_history else None))
    if not want_history:
        return None
    return hist[:n_iter, 0] if nc == 1 else hist[:n_iter]


def ql_step_static(s, n_iter, want_history=True):
    """ql_step with its residual history in the library's fixed device
    array (no device allocation); same return value as ql_step."""
    nc = ql_batch_info(s)
    hist = np.zeros((max(int(n_iter), 1), nc, 4))
    _check(s, lib.ql_step_static(s, int(n_iter), hist.ctypes.data if want_history else None))
    if not want_history:
        return None
    return hist[:n_iter, 0] if nc == 1 else hist[:n_iter]


def ql_batch_upload(s, case_ptr, x, y, nx, ny, kind, nbr_ptr, nbr_idx, mach, alpha_deg):
    cp = np.ascontiguousarray(case_ptr, dtype=np.int64)
    keep = [_host(x, np.float64), _host(y, np.float64), _host(nx, np.float64),
            _host(ny, np.float64), _host(kind, np.uint8), _host(nbr_ptr, np.int32),
            _host(nbr_idx, np.int32)]
    m = np.ascontiguousarray(mach, dtype=np.float64)
    a = np.ascontiguousarray(alpha_deg, dtype=np.float64)
    n = keep[0][0].shape[0]
    return _check(s, lib.ql_batch_upload(s, cp.shape[0] - 1, cp.ctypes.data, n,
                                         *(k[1] for k in keep), m.ctypes.data, a.ctypes.data))


def ql_batch_run(s, drop, max_iter, check_every=100, graph=True, ref=None):
    """Returns (iterations per case, last residual norms (ncase, 4)); ref:
    per-case reference density-residual norms (None: first iteration's)."""
    nc = ql_batch_info(s)
    iters = np.zeros(nc, np.int32)
    res = np.zeros((nc, 4))
    keep = None
    if ref is not None:
        keep = np.ascontiguousarray(ref, dtype=np.float64)
        if keep.shape != (nc,):
            raise ValueError("ref must hold one value per case")
    _check(s, lib.ql_batch_run(s, float(drop), int(max_iter), int(check_every), int(bool(graph)),
                               keep.ctypes.data if keep is not None else None,
                               iters.ctypes.data, res.ctypes.data))
    return iters, res


def ql_batch_status(s):
    """Per-case status of the last ql_batch_run (QL_OK, or the failure code
    of a case that was retired)."""
    out = np.zeros(ql_batch_info(s), np.int32)
    _check(s, lib.ql_batch_status(s, out.ctypes.data))
    return out


def ql_batch_switched(s):
    """Per case, the iteration of the last ql_batch_run after which it moved
    from FP32 to FP64 split fluxes (-1: never)."""
    out = np.zeros(ql_batch_info(s), np.int32)
    _check(s, lib.ql_batch_switched(s, out.ctypes.data))
    return out


def ql_set_progress(s, fn):
    """fn(iterations, active) after every check window of ql_batch_run, or
    None; returns the ctypes callback, which must stay referenced while it
    is set."""
    cb = PROGRESS_FN(lambda _user, it, active: fn(int(it), int(active))) if fn else \
        C.cast(None, PROGRESS_FN)
    _check(s, lib.ql_set_progress(s, cb, None))
    return cb


def ql_autotune(s, cache_path=None):
    """Tune the LDS budgets on the current state; returns (flux_lds, grad_lds)."""
    out = np.zeros(2, np.int32)
    _check(s, lib.ql_autotune(s, cache_path.encode() if cache_path else None,
                              out.ctypes.data))
    return int(out[0]), int(out[1])


def ql_wall_distance(s):
    n, _ = ql_cloud_size(s)
    out = np.empty(n)
    _check(s, lib.ql_wall_distance(s, out.ctypes.data))
    return out


def ql_warm_start(s, m, X, out_scale, rel_floor=0.05):
    """X: device float32 tensor (n, w_in) in caller order; out_scale: 8
    floats (mean[4], std[4]).  Returns (res_cold (ncase, 4), res_warm
    (ncase, 4), used (ncase,) bool)."""
    nc = ql_batch_info(s)
    sc = np.ascontiguousarray(out_scale, dtype=np.float32)
    if sc.shape != (8,):
        raise ValueError("out_scale must hold 8 values")
    rc, rw = np.zeros((nc, 4)), np.zeros((nc, 4))
    used = np.zeros(nc, np.int32)
    _check(s, lib.ql_warm_start(s, m, _dev_ptr(X), sc.ctypes.data, float(rel_floor),
                                rc.ctypes.data, rw.ctypes.data, used.ctypes.data))
    return rc, rw, used.astype(bool)


# --- warm-start network --------------------------------------------------

def _mcheck(m, rc):
    if rc != QL_OK:
        msg = lib.ql_mlp_last_error(m).decode() if m else ""
        raise QLError(rc, msg)
    return rc


def ql_mlp_create(widths, max_batch, device=0, stream=None):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
    elif not isinstance(stream, int):
        stream = stream.cuda_stream
    w = np.ascontiguousarray(widths, dtype=np.int32)
    h = C.c_void_p()
    rc = lib.ql_mlp_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None,
                           w.ctypes.data, int(w.size), int(max_batch))
    if rc != QL_OK:
        raise QLError(rc, "ql_mlp_create failed")
    return h


def ql_mlp_destroy(m):
    return lib.ql_mlp_destroy(m)


def ql_mlp_num_params(m):
    n = C.c_int64()
    _mcheck(m, lib.ql_mlp_num_params(m, C.byref(n)))
    return n.value


def ql_mlp_set_weights(m, w):
    a = np.ascontiguousarray(w, dtype=np.float32)
    if a.size != ql_mlp_num_params(m):
        raise ValueError("weight vector has the wrong length")
    return _mcheck(m, lib.ql_mlp_set_weights(m, a.ctypes.data))


def ql_mlp_get_weights(m):
    out = np.empty(ql_mlp_num_params(m), np.float32)
    _mcheck(m, lib.ql_mlp_get_weights(m, out.ctypes.data))
    return out


def ql_mlp_forward(m, X, Y, n):
    return _mcheck(m, lib.ql_mlp_forward(m, _dev_ptr(X), _dev_ptr(Y), int(n)))


def ql_mlp_gradient(m, X, T, n):
    """(loss, gradient as float32[np])."""
    g = np.empty(ql_mlp_num_params(m), np.float32)
    loss = C.c_double()
    _mcheck(m, lib.ql_mlp_gradient(m, _dev_ptr(X), _dev_ptr(T), int(n), g.ctypes.data,
                                   C.byref(loss)))
    return loss.value, g


def ql_mlp_train_step(m, X, T, n, lr, want_loss=True):
    loss = C.c_double()
    _mcheck(m, lib.ql_mlp_train_step(m, _dev_ptr(X), _dev_ptr(T), int(n), float(lr),
                                     C.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def ql_mlp_sync(m):
    return _mcheck(m, lib.ql_mlp_sync(m))


class Mlp:
    """Convenience owner of one network handle."""

    def __init__(self, widths, max_batch, device=0, stream=None):
        self.widths = list(widths)
        self.h = ql_mlp_create(widths, max_batch, device, stream)

    @property
    def num_params(self):
        return ql_mlp_num_params(self.h)

    def set_weights(self, w):
        ql_mlp_set_weights(self.h, w)

    def get_weights(self):
        return ql_mlp_get_weights(self.h)

    def _rows(self, X, width):
        import torch
        if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != width:
            raise ValueError(f"expected a float32 (n, {width}) tensor")
        return X.shape[0]

    def forward(self, X, Y=None):
        import torch
        self._rows(X, self.widths[0])
        if Y is None:
            Y = torch.empty((X.shape[0], self.widths[-1]), dtype=torch.float32, device=X.device)
        ql_mlp_forward(self.h, X, Y, X.shape[0])
        ql_mlp_sync(self.h)
        return Y

    def gradient(self, X, T):
        n = self._rows(X, self.widths[0])
        if self._rows(T, self.widths[-1]) != n:
            raise ValueError("X and T must have the same rows")
        return ql_mlp_gradient(self.h, X, T, n)

    def train_step(self, X, T, lr, want_loss=True):
        n = self._rows(X, self.widths[0])
        if self._rows(T, self.widths[-1]) != n:
            raise ValueError("X and T must have the same rows")
        return ql_mlp_train_step(self.h, X, T, n, lr, want_loss)

    def close(self):
        if self.h:
            ql_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ql_batch_forces(s):
    nc = ql_batch_info(s)
    cl, cd = np.zeros(nc), np.zeros(nc)
    _check(s, lib.ql_batch_forces(s, cl.ctypes.data, cd.ctypes.data))
    return cl, cd


def ql_residual_norm(s):
    out = np.zeros(4)
    _check(s, lib.ql_residual_norm(s, out.ctypes.data))
    return out


def ql_cloud_size(s):
    n, nnz = C.c_int64(), C.c_int64()
    _check(s, lib.ql_cloud_size(s, C.byref(n), C.byref(nnz)))
    return n.value, nnz.value


def ql_fetch_state(s, out=None):
    """Into a new host array (4, n), or into `out` (numpy or torch CUDA)."""
    n, _ = ql_cloud_size(s)
    if out is None:
        out = np.empty((4, n))
    if isinstance(out, np.ndarray):
        if out.dtype != np.float64 or not out.flags.c_contiguous or out.shape != (4, n):
            raise ValueError("out must be C-contiguous float64 (4, n)")
        _check(s, lib.ql_fetch_state(s, out.ctypes.data, 0))
    else:
        _check(s, lib.ql_fetch_state(s, _dev_ptr(out), 1))
    return out


def ql_forces(s):
    cl, cd = C.c_double(), C.c_double()
    _check(s, lib.ql_forces(s, C.byref(cl), C.byref(cd)))
    return cl.value, cd.value


def ql_last_error(s):
    return lib.ql_last_error(s).decode()


def ql_evaluate(s):
    return _check(s, lib.ql_evaluate(s))


_DEBUG_ROWS = {0: 4, 1: 8, 2: 4, 3: 1, 4: 4, 5: 4}


def ql_debug_fetch(s, what):
    n, _ = ql_cloud_size(s)
    rows = _DEBUG_ROWS[what]
    out = np.empty((rows, n)) if rows > 1 else np.empty(n)
    _check(s, lib.ql_debug_fetch(s, int(what), out.ctypes.data))
    return out


def ql_flux_tiles(s):
    """Records in each flux tile's LDS image, int32[ntile]."""
    nt = C.c_int32()
    _check(s, lib.ql_flux_tiles(s, C.byref(nt), None))
    out = np.empty(nt.value, np.int32)
    _check(s, lib.ql_flux_tiles(s, C.byref(nt), out.ctypes.data))
    return out


def ql_debug_flags(s):
    _, nnz = ql_cloud_size(s)
    out = np.empty(nnz, np.uint8)
    _check(s, lib.ql_debug_flags(s, out.ctypes.data))
    return out


def ql_set_timing(s, enable):
    return _check(s, lib.ql_set_timing(s, int(bool(enable))))


def ql_kernel_time(s, which):
    ms, cnt = C.c_double(), C.c_int64()
    _check(s, lib.ql_kernel_time(s, int(which), C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


def params(**kw):
    """ql_params with defaults overridden by keyword."""
    p = ql_default_params()
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Solver:
    """Convenience owner of one solver handle (same calls, bound)."""

    def __init__(self, cloud=None, device=0, stream=None, **prm):
        self.h = ql_create(device, stream)
        self._prm = dict(prm)
        if prm:
            ql_set_params(self.h, params(**prm))
        if cloud is not None:
            self.upload(cloud)

    def upload_batch(self, clouds, mach, alpha_deg):
        """Concatenate independent clouds into one batched upload."""
        offs = np.cumsum([0] + [c.n for c in clouds])
        eoffs = np.cumsum([0] + [c.nnz for c in clouds])
        cat = lambda f: np.concatenate([getattr(c, f) for c in clouds])
        ptr = np.concatenate([c.nbr_ptr[:-1].astype(np.int64) + e for c, e in zip(clouds, eoffs)]
                             + [np.array([eoffs[-1]])])
        idx = np.concatenate([c.nbr_idx.astype(np.int64) + o for c, o in zip(clouds, offs)])
        ql_batch_upload(self.h, offs, cat("x"), cat("y"), cat("nx"), cat("ny"), cat("kind"),
                        ptr, idx, mach, alpha_deg)
        return offs

    def batch_run(self, drop, max_iter, check_every=100, graph=True, ref=None):
        return ql_batch_run(self.h, drop, max_iter, check_every, graph, ref)

    def batch_status(self):
        return ql_batch_status(self.h)

    def batch_switched(self):
        return ql_batch_switched(self.h)

    def set_progress(self, fn):
        """fn(iterations, active) after every check window of batch_run."""
        self._progress = ql_set_progress(self.h, fn)

    def wall_distance(self):
        return ql_wall_distance(self.h)

    def autotune(self, cache_path=None):
        f, g = ql_autotune(self.h, cache_path)
        self._prm.update(flux_lds=f, grad_lds=g)
        return f, g

    def warm_start(self, mlp, X, out_scale, rel_floor=0.05):
        n, _ = ql_cloud_size(self.h)
        if mlp._rows(X, mlp.widths[0]) != n:
            raise ValueError("one feature row per point is needed")
        return ql_warm_start(self.h, mlp.h, X, out_scale, rel_floor)

    def batch_forces(self):
        return ql_batch_forces(self.h)

    def upload(self, cloud, nbr_flag=None):
        ql_upload_cloud(self.h, cloud.x, cloud.y, cloud.nx, cloud.ny, cloud.kind,
                        cloud.nbr_ptr, cloud.nbr_idx, nbr_flag)

    def set_params(self, **prm):
        """Change the given parameters, keeping the others."""
        merged = dict(self._prm, **prm)
        ql_set_params(self.h, params(**merged))
        self._prm = merged

    def init_freestream(self):
        ql_init_freestream(self.h)

    def set_state(self, U, project_wall=False):
        ql_set_state(self.h, U, project_wall)

    def step(self, n_iter, want_history=True):
        return ql_step(self.h, n_iter, want_history)

    def step_static(self, n_iter, want_history=True):
        return ql_step_static(self.h, n_iter, want_history)

    def residual_norm(self):
        return ql_residual_norm(self.h)

    def fetch_state(self, out=None):
        return ql_fetch_state(self.h, out)

    def forces(self):
        return ql_forces(self.h)

    def evaluate(self):
        ql_evaluate(self.h)
        return {name: ql_debug_fetch(self.h, w) for w, name in
                enumerate(("q", "g", "R", "dt", "qmax", "qmin"))}

    def flags(self):
        return ql_debug_flags(self.h)

    def flux_tiles(self):
        return ql_flux_tiles(self.h)

    def close(self):
        if self.h:
            ql_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
