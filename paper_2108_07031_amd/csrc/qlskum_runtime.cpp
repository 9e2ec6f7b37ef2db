// Host runtime of the q-LSKUM solver: the C ABI of include/qlskum.h.
//
// Owns the device buffers of one solver, validates and reorders the point
// cloud, and drives the kernels of one pseudo-time iteration (sec. 3,
// Algorithm 1): per stage the gradient first pass, n_inner inner
// iterations and the fused flux-residual + Runge-Kutta-stage kernel; per
// iteration one residual-norm reduction.  All compute runs in the kernels
// of qlskum_kernels.hip; the host only validates, permutes indices and
// enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/qlskum.h"
#include "qlskum_internal.h"

using namespace ql;

namespace {

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
};

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

struct ql_solver {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    std::string err;
    ql_params prm{};

    // cloud (library order)
    int n = 0;
    int64_t nnz = 0;
    int n_upd = 0;
    bool has_cloud = false, has_state = false, has_eval = false, has_res = false;
    std::vector<int> perm;       // library point -> caller point
    std::vector<int> inv;        // caller point -> library point
    std::vector<int64_t> eperm;  // library entry -> caller entry
    int nw = 0;

    double2 *xy = nullptr, *nrm = nullptr;
    uint8_t *kind = nullptr, *flag = nullptr;
    int *ptr = nullptr, *idx = nullptr, *dperm = nullptr, *wall = nullptr;
    double *lsw = nullptr, *dmin = nullptr;
    double *U = nullptr, *Un = nullptr, *dt = nullptr, *R = nullptr, *tmp = nullptr;
    double2 *q[2] = {nullptr, nullptr}, *g[3] = {nullptr, nullptr, nullptr}, *qmm = nullptr;
    float4 *q32[2] = {nullptr, nullptr}, *g32 = nullptr, *qmm32 = nullptr;  // FP32 shadows
    int *halo_ptr = nullptr, *halo_idx = nullptr;
    uint16_t *lidx = nullptr;
    int max_slots = 0;
    double *partial = nullptr, *reshist = nullptr, *fscratch = nullptr, *fout = nullptr;
    int reshist_cap = 0;
    int *errw = nullptr;
    int err_init[2] = {INT_MAX, 0};  // source of the error-word reset copies
    int qcur = 0, gfin = 0;
    double last_res[4] = {0, 0, 0, 0};

    bool timing = false;
    bool untiled = false;  // QLSKUM_UNTILED=1: gather straight from memory (A/B checks)
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    double tsum[4] = {0, 0, 0, 0};
    int64_t tcnt[4] = {0, 0, 0, 0};
};

namespace {

int fail(ql_solver *s, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s->err = buf;
    if (code == QL_EDEVICE) s->poisoned = true;
    return code;
}

#define HIPCHK(s, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((s), QL_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_cloud(ql_solver *s) {
    dfree(s->xy); dfree(s->nrm); dfree(s->kind); dfree(s->flag); dfree(s->ptr); dfree(s->idx);
    dfree(s->dperm); dfree(s->wall); dfree(s->lsw); dfree(s->dmin); dfree(s->U); dfree(s->Un);
    dfree(s->dt); dfree(s->R); dfree(s->tmp); dfree(s->q[0]); dfree(s->q[1]); dfree(s->g[0]);
    dfree(s->g[1]); dfree(s->g[2]); dfree(s->qmm); dfree(s->partial); dfree(s->reshist);
    dfree(s->fscratch); dfree(s->fout); dfree(s->errw); dfree(s->halo_ptr); dfree(s->halo_idx);
    dfree(s->lidx); dfree(s->q32[0]); dfree(s->q32[1]); dfree(s->g32); dfree(s->qmm32);
    s->max_slots = 0;
    s->reshist_cap = 0;
    s->has_cloud = s->has_state = s->has_eval = s->has_res = false;
    s->n = 0;
    s->nnz = 0;
}

// Hilbert index of (x, y) on a 2^order x 2^order grid (order <= 31).
uint64_t hilbert_key(uint32_t x, uint32_t y, int order) {
    uint64_t d = 0;
    const uint32_t full = (order >= 32) ? 0xffffffffu : ((1u << order) - 1u);
    for (uint32_t sbit = 1u << (order - 1); sbit > 0; sbit >>= 1) {
        const uint32_t rx = (x & sbit) ? 1u : 0u;
        const uint32_t ry = (y & sbit) ? 1u : 0u;
        d += (uint64_t)sbit * (uint64_t)sbit * (uint64_t)((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x ^= full;
                y ^= full;
            }
            std::swap(x, y);
        }
    }
    return d;
}

std::vector<int> hilbert_order(int n, const double *x, const double *y) {
    double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
    for (int p = 1; p < n; ++p) {
        x0 = std::min(x0, x[p]); x1 = std::max(x1, x[p]);
        y0 = std::min(y0, y[p]); y1 = std::max(y1, y[p]);
    }
    const int order = 31;
    const double span = std::max(x1 - x0, y1 - y0);
    const double scale = (span > 0.0) ? (double)((1u << order) - 1u) / span : 0.0;
    std::vector<uint64_t> key(n);
    for (int p = 0; p < n; ++p) {
        const uint32_t qx = (uint32_t)std::min((x[p] - x0) * scale, (double)((1u << order) - 1u));
        const uint32_t qy = (uint32_t)std::min((y[p] - y0) * scale, (double)((1u << order) - 1u));
        key[p] = hilbert_key(qx, qy, order);
    }
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int a, int b) { return key[a] < key[b]; });
    return perm;
}

// Tiles of kBlock consecutive points: the sorted list of each tile's halo
// (neighbours outside the tile) and every entry's slot in the tile's LDS
// image.  Returns the largest image (own slots + halo), or INT_MAX when a
// slot would not fit 16 bits.
int build_tiles(int n, const std::vector<int> &ptr, const std::vector<int> &idx,
                std::vector<int> &hptr, std::vector<int> &hidx, std::vector<uint16_t> &lidx) {
    const int ntile = num_blocks(n);
    hptr.assign(ntile + 1, 0);
    hidx.clear();
    lidx.assign(idx.size(), 0);
    std::vector<int> stamp(n, -1), slot(n, 0), h;
    int max_slots = 0;
    for (int t = 0; t < ntile; ++t) {
        const int base = t * kBlock, end = std::min(n, base + kBlock);
        h.clear();
        for (int p = base; p < end; ++p)
            for (int k = ptr[p]; k < ptr[p + 1]; ++k) {
                const int i = idx[k];
                if ((i < base || i >= end) && stamp[i] != t) {
                    stamp[i] = t;
                    h.push_back(i);
                }
            }
        std::sort(h.begin(), h.end());
        const int slots = kBlock + (int)h.size();
        if (slots > 65535) return INT_MAX;
        for (size_t j = 0; j < h.size(); ++j) slot[h[j]] = kBlock + (int)j;
        for (int p = base; p < end; ++p)
            for (int k = ptr[p]; k < ptr[p + 1]; ++k) {
                const int i = idx[k];
                lidx[k] = (uint16_t)((i >= base && i < end) ? i - base : slot[i]);
            }
        hidx.insert(hidx.end(), h.begin(), h.end());
        hptr[t + 1] = (int)hidx.size();
        max_slots = std::max(max_slots, slots);
    }
    return max_slots;
}

DevCloud dev_cloud(const ql_solver *s) {
    DevCloud c;
    c.n = s->n;
    c.xy = s->xy;
    c.nrm = s->nrm;
    c.kind = s->kind;
    c.ptr = s->ptr;
    c.idx = s->idx;
    c.flag = s->flag;
    c.lsw = s->lsw;
    c.dmin = s->dmin;
    c.halo_ptr = s->halo_ptr;
    c.halo_idx = s->halo_idx;
    c.lidx = s->lidx;
    c.max_slots = s->max_slots;
    return c;
}

FlowParams flow_params(const ql_solver *s) {
    FlowParams f;
    f.gamma = s->prm.gamma;
    f.gm1inv = 1.0 / (s->prm.gamma - 1.0);
    f.cfl = s->prm.cfl;
    f.venkat_k = s->prm.venkat_k;
    f.n_inner = s->prm.n_inner;
    f.limiter = s->prm.limiter;
    const double m = 2.0 / (s->prm.gamma - 1.0);
    const double mr = std::nearbyint(m);
    f.sqrt_pow = (std::fabs(m - mr) <= 1e-12 * m && mr >= 1.0 && mr <= 16.0) ? (int)mr : 0;
    return f;
}

int check_params(ql_solver *s, const ql_params *p) {
    if (!p) return fail(s, QL_EINVAL, "params is NULL");
    if (!(p->gamma > 1.0 && p->gamma < 2.0)) return fail(s, QL_EINVAL, "gamma must be in (1, 2)");
    if (!(p->mach >= 0.0) || !std::isfinite(p->mach)) return fail(s, QL_EINVAL, "bad mach");
    if (!std::isfinite(p->alpha_deg)) return fail(s, QL_EINVAL, "bad alpha");
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return fail(s, QL_EINVAL, "cfl must be > 0");
    if (p->n_inner < 0 || p->n_inner > 1000) return fail(s, QL_EINVAL, "n_inner out of range");
    if (p->limiter != 0 && p->limiter != 1) return fail(s, QL_EINVAL, "limiter must be 0 or 1");
    if (p->limiter && !(p->venkat_k > 0.0)) return fail(s, QL_EINVAL, "venkat_k must be > 0");
    if (p->precision != 0 && p->precision != 1)
        return fail(s, QL_EINVAL, "precision must be 0 (FP64) or 1 (mixed)");
    if (p->reorder != 0 && p->reorder != 1) return fail(s, QL_EINVAL, "reorder must be 0 or 1");
    return QL_OK;
}

int reset_err(ql_solver *s) {
    HIPCHK(s, hipMemcpyAsync(s->errw, s->err_init, sizeof s->err_init, hipMemcpyHostToDevice,
                             s->stream));
    return QL_OK;
}

// Synchronise and turn the device error word into a status.
int sync_and_check(ql_solver *s, const char *what) {
    int e[2];
    HIPCHK(s, hipMemcpyAsync(e, s->errw, sizeof e, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (e[1] == kErrNone) return QL_OK;
    const int up = (e[0] >= 0 && e[0] < s->n) ? s->perm[e[0]] : -1;
    switch (e[1]) {
    case kErrSingular:
        return fail(s, QL_ESINGULAR, "%s: singular least-squares stencil at point %d", what, up);
    case kErrNonFinite:
        return fail(s, QL_ENONFINITE, "%s: non-finite state at point %d", what, up);
    default:
        return fail(s, QL_EPOSITIVITY,
                    "%s: positivity lost (non-positive density/pressure or q4 >= 0) at point %d",
                    what, up);
    }
}

hipEvent_t take_event(ql_solver *s) {
    hipEvent_t e = nullptr;
    if (!s->event_pool.empty()) {
        e = s->event_pool.back();
        s->event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Collect the timed launches after a synchronisation.
void harvest_timing(ql_solver *s) {
    for (auto &t : s->pending) {
        float ms = 0.0f;
        if (t.a && t.b && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            s->tsum[t.kind] += ms;
            s->tcnt[t.kind] += 1;
        }
        if (t.a) s->event_pool.push_back(t.a);
        if (t.b) s->event_pool.push_back(t.b);
    }
    s->pending.clear();
}

struct Timer {
    ql_solver *s;
    int kind;
    hipEvent_t a = nullptr;
    Timer(ql_solver *s_, int k) : s(s_), kind(k) {
        if (s->timing) {
            a = take_event(s);
            if (a) (void)hipEventRecord(a, s->stream);
        }
    }
    void done() {
        if (s->timing && a) {
            hipEvent_t b = take_event(s);
            if (b) (void)hipEventRecord(b, s->stream);
            s->pending.push_back({kind, a, b});
        }
    }
};

// One stage's q-derivatives: first pass + n_inner Jacobi iterations; leaves
// the final iterate in g[gfin].
int run_gradients(ql_solver *s, const DevCloud &c, bool want_bounds) {
    const bool tiled = !s->untiled;
    const bool lds0 = tiled && lds_fits_grad0(c), ldsk = tiled && lds_fits_gradk(c);
    // first pass into g[2] when the inner iterations run tiled (they read g0)
    const int first = (ldsk && s->prm.n_inner > 0) ? 2 : 0;
    // mixed precision: the last pass also writes the FP32 shadow of g, the
    // first pass the FP32 shadow of the bounds
    const bool mixed = s->prm.precision == 1;
    Shadow sh{nullptr, nullptr, nullptr};
    if (mixed) {
        sh.qmm32 = s->qmm32;
        if (s->prm.n_inner == 0) sh.g32 = s->g32;
    }
    {
        Timer t(s, 0);
        if (lds0)
            HIPCHK(s, launch_grad0_lds(s->stream, c, s->q[s->qcur], s->g[first], s->qmm,
                                       want_bounds ? 1 : 0, sh));
        else
            HIPCHK(s, launch_grad0(s->stream, c, s->q[s->qcur], s->g[first], s->qmm,
                                   want_bounds ? 1 : 0, sh));
        t.done();
    }
    int cur = first;
    for (int k = 0; k < s->prm.n_inner; ++k) {
        const int nxt = (cur == 0) ? 1 : 0;
        float4 *g32 = (mixed && k == s->prm.n_inner - 1) ? s->g32 : nullptr;
        Timer t(s, 1);
        if (ldsk)
            HIPCHK(s, launch_gradk_lds(s->stream, c, s->g[2], s->g[cur], s->g[nxt], g32));
        else
            HIPCHK(s, launch_gradk(s->stream, c, s->q[s->qcur], s->g[cur], s->g[nxt], g32));
        t.done();
        cur = nxt;
    }
    s->gfin = cur;
    return QL_OK;
}

// Enqueue q and the time step of the current state (start of an iteration).
int prep_state(ql_solver *s) {
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    int st = reset_err(s);
    if (st) return st;
    s->qcur = 0;
    HIPCHK(s, launch_prep(s->stream, c, fp, s->U, s->Un, s->q[0], s->dt, s->q32[0], s->errw));
    return QL_OK;
}

// One flux-residual launch (stage 0: evaluate into R; 1..4: RK stage).
int launch_stage(ql_solver *s, const DevCloud &c, const FlowParams &fp, int stage, double *Rout,
                 double *partial) {
    const int a = s->qcur, b = 1 - s->qcur;
    if (s->prm.precision == 1)
        HIPCHK(s, launch_flux_mixed(s->stream, c, fp, stage, s->q[a], s->q32[a], s->g32, s->qmm32,
                                    s->U, s->Un, s->dt, s->q[b], s->q32[b], Rout, partial,
                                    s->errw));
    else
        HIPCHK(s, launch_flux(s->stream, c, fp, stage, s->q[a], s->g[s->gfin], s->qmm, s->U,
                              s->Un, s->dt, s->q[b], Rout, partial, s->q32[b], s->errw));
    return QL_OK;
}

int ensure_ready(ql_solver *s, bool need_state) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    if (!s->has_cloud) return fail(s, QL_ESTATE, "no cloud uploaded");
    if (need_state && !s->has_state) return fail(s, QL_ESTATE, "no flow state set");
    return QL_OK;
}

}  // namespace

extern "C" {

void ql_default_params(ql_params *p) {
    if (!p) return;
    p->gamma = 1.4;
    p->mach = 0.63;
    p->alpha_deg = 2.0;
    p->cfl = 0.2;
    p->n_inner = 3;
    p->limiter = 0;
    p->venkat_k = 5.0;
    p->precision = 0;
    p->reorder = 1;
}

int ql_create(ql_solver **out, int32_t device, void *hip_stream) {
    if (!out) return QL_EINVAL;
    *out = nullptr;
    ql_solver *s = new (std::nothrow) ql_solver();
    if (!s) return QL_ENOMEM;
    ql_default_params(&s->prm);
    s->device = device;
    if (const char *e = std::getenv("QLSKUM_UNTILED")) s->untiled = (e[0] == '1');
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete s;
        return QL_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete s;
        return QL_EDEVICE;
    }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) {
            delete s;
            return QL_EDEVICE;
        }
        s->own_stream = true;
    }
    *out = s;
    return QL_OK;
}

int ql_destroy(ql_solver *s) {
    if (!s) return QL_OK;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_cloud(s);
    for (auto &t : s->pending) {
        if (t.a) (void)hipEventDestroy(t.a);
        if (t.b) (void)hipEventDestroy(t.b);
    }
    for (auto e : s->event_pool) (void)hipEventDestroy(e);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return QL_OK;
}

const char *ql_last_error(const ql_solver *s) { return s ? s->err.c_str() : "null solver"; }

int ql_set_params(ql_solver *s, const ql_params *p) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    int st = check_params(s, p);
    if (st) return st;
    s->prm = *p;
    return QL_OK;
}

int ql_upload_cloud(ql_solver *s, int64_t n64, const double *x, const double *y,
                    const double *nx, const double *ny, const uint8_t *kind,
                    const int32_t *nbr_ptr, const int32_t *nbr_idx, const uint8_t *nbr_flag) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    if (!x || !y || !nx || !ny || !kind || !nbr_ptr || (!nbr_idx && n64 > 0))
        return fail(s, QL_EINVAL, "null array argument");
    if (n64 < 1 || n64 > INT_MAX / 8) return fail(s, QL_EINVAL, "n = %lld out of range", (long long)n64);
    const int n = (int)n64;
    if (nbr_ptr[0] != 0) return fail(s, QL_EINVAL, "nbr_ptr[0] must be 0");
    for (int p = 0; p < n; ++p) {
        if (nbr_ptr[p + 1] < nbr_ptr[p]) return fail(s, QL_EINVAL, "nbr_ptr decreases at point %d", p);
        if (kind[p] > QL_KIND_OUTER) return fail(s, QL_EINVAL, "bad kind %d at point %d", kind[p], p);
        if (!std::isfinite(x[p]) || !std::isfinite(y[p]))
            return fail(s, QL_EINVAL, "non-finite coordinate at point %d", p);
        const double nn = nx[p] * nx[p] + ny[p] * ny[p];
        if (!(std::fabs(nn - 1.0) < 1e-8)) return fail(s, QL_EINVAL, "normal of point %d is not unit", p);
    }
    const int64_t nnz = nbr_ptr[n];
    for (int p = 0; p < n; ++p)
        for (int k = nbr_ptr[p]; k < nbr_ptr[p + 1]; ++k) {
            const int i = nbr_idx[k];
            if (i < 0 || i >= n || i == p)
                return fail(s, QL_EINVAL, "neighbour entry %d of point %d is out of range or self", k, p);
            if (nbr_flag && (nbr_flag[k] & ~0x0f))
                return fail(s, QL_EINVAL, "bad split flag at entry %d", k);
        }
    (void)hipSetDevice(s->device);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    free_cloud(s);

    // point order
    std::vector<int> perm;
    if (s->prm.reorder == 1) perm = hilbert_order(n, x, y);
    else { perm.resize(n); std::iota(perm.begin(), perm.end(), 0); }
    std::vector<int> inv(n);
    for (int q = 0; q < n; ++q) inv[perm[q]] = q;

    // reordered host arrays
    std::vector<double2> hxy(n), hnrm(n);
    std::vector<uint8_t> hkind(n), hflag(nbr_flag ? nnz : 0);
    std::vector<int> hptr(n + 1), hidx(nnz);
    std::vector<int64_t> eperm(nnz);
    hptr[0] = 0;
    for (int q = 0; q < n; ++q) {
        const int p = perm[q];
        hxy[q] = make_double2(x[p], y[p]);
        hnrm[q] = make_double2(nx[p], ny[p]);
        hkind[q] = kind[p];
        int k = hptr[q];
        for (int e = nbr_ptr[p]; e < nbr_ptr[p + 1]; ++e, ++k) {
            hidx[k] = inv[nbr_idx[e]];
            eperm[k] = e;
            if (nbr_flag) hflag[k] = nbr_flag[e];
        }
        hptr[q + 1] = k;
    }
    std::vector<int> hwall;
    int n_upd = 0;
    for (int p = 0; p < n; ++p) {
        if (kind[p] == QL_KIND_WALL) hwall.push_back(inv[p]);
        if (kind[p] != QL_KIND_OUTER) ++n_upd;
    }
    const int nblk = num_blocks(n);

    s->n = n;
    s->nnz = nnz;
    s->n_upd = n_upd;
    s->nw = (int)hwall.size();
    HIPCHK(s, dalloc(&s->xy, n)); HIPCHK(s, dalloc(&s->nrm, n)); HIPCHK(s, dalloc(&s->kind, n));
    HIPCHK(s, dalloc(&s->flag, nnz)); HIPCHK(s, dalloc(&s->ptr, n + 1)); HIPCHK(s, dalloc(&s->idx, nnz));
    HIPCHK(s, dalloc(&s->dperm, n)); HIPCHK(s, dalloc(&s->wall, hwall.size()));
    HIPCHK(s, dalloc(&s->lsw, (size_t)8 * n)); HIPCHK(s, dalloc(&s->dmin, n));
    HIPCHK(s, dalloc(&s->U, (size_t)4 * n)); HIPCHK(s, dalloc(&s->Un, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->dt, n)); HIPCHK(s, dalloc(&s->R, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->tmp, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->q[0], (size_t)2 * n)); HIPCHK(s, dalloc(&s->q[1], (size_t)2 * n));
    HIPCHK(s, dalloc(&s->g[0], (size_t)4 * n)); HIPCHK(s, dalloc(&s->g[1], (size_t)4 * n));
    HIPCHK(s, dalloc(&s->g[2], (size_t)4 * n));
    HIPCHK(s, dalloc(&s->qmm, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->q32[0], n)); HIPCHK(s, dalloc(&s->q32[1], n));
    HIPCHK(s, dalloc(&s->g32, (size_t)2 * n)); HIPCHK(s, dalloc(&s->qmm32, (size_t)2 * n));
    HIPCHK(s, dalloc(&s->partial, (size_t)4 * nblk));
    HIPCHK(s, dalloc(&s->fscratch, (size_t)3 * std::max<size_t>(hwall.size(), 1)));
    HIPCHK(s, dalloc(&s->fout, 2)); HIPCHK(s, dalloc(&s->errw, 2));

    hipStream_t st = s->stream;
    HIPCHK(s, hipMemcpyAsync(s->xy, hxy.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->nrm, hnrm.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->kind, hkind.data(), n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->ptr, hptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
    if (nnz) HIPCHK(s, hipMemcpyAsync(s->idx, hidx.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, st));
    if (nbr_flag && nnz) HIPCHK(s, hipMemcpyAsync(s->flag, hflag.data(), nnz, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->dperm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    if (!hwall.empty())
        HIPCHK(s, hipMemcpyAsync(s->wall, hwall.data(), sizeof(int) * hwall.size(), hipMemcpyHostToDevice, st));
    {
        std::vector<int> thptr, thidx;
        std::vector<uint16_t> tlidx;
        s->max_slots = build_tiles(n, hptr, hidx, thptr, thidx, tlidx);
        if (s->max_slots == INT_MAX) {
            s->max_slots = 1 << 30;  // no tiled kernels for this cloud
        } else {
            HIPCHK(s, dalloc(&s->halo_ptr, thptr.size()));
            HIPCHK(s, dalloc(&s->halo_idx, thidx.size()));
            HIPCHK(s, dalloc(&s->lidx, tlidx.size()));
            HIPCHK(s, hipMemcpy(s->halo_ptr, thptr.data(), sizeof(int) * thptr.size(),
                                hipMemcpyHostToDevice));
            if (!thidx.empty())
                HIPCHK(s, hipMemcpy(s->halo_idx, thidx.data(), sizeof(int) * thidx.size(),
                                    hipMemcpyHostToDevice));
            if (!tlidx.empty())
                HIPCHK(s, hipMemcpy(s->lidx, tlidx.data(), sizeof(uint16_t) * tlidx.size(),
                                    hipMemcpyHostToDevice));
        }
    }
    s->perm.swap(perm);
    s->inv.swap(inv);
    s->eperm.swap(eperm);

    int rc = reset_err(s);
    if (rc) return rc;
    HIPCHK(s, launch_setup(st, n, s->xy, s->nrm, s->kind, s->ptr, s->idx, s->flag,
                           nbr_flag ? 0 : 1, s->lsw, s->dmin, s->errw));
    // host buffers above must outlive the asynchronous copies
    rc = sync_and_check(s, "upload");
    if (rc) {
        const std::string msg = s->err;
        free_cloud(s);
        s->err = msg;
        return rc;
    }
    s->has_cloud = true;
    return QL_OK;
}

int ql_cloud_size(const ql_solver *s, int64_t *n, int64_t *nnz) {
    if (!s || !s->has_cloud) return QL_ESTATE;
    if (n) *n = s->n;
    if (nnz) *nnz = s->nnz;
    return QL_OK;
}

int ql_init_freestream(ql_solver *s) {
    int st = ensure_ready(s, false);
    if (st) return st;
    (void)hipSetDevice(s->device);
    const double a = s->prm.alpha_deg * M_PI / 180.0;
    const double rho = 1.0, u1 = s->prm.mach * std::cos(a), u2 = s->prm.mach * std::sin(a);
    const double p = 1.0 / s->prm.gamma;
    const double Uinf[4] = {rho, rho * u1, rho * u2,
                            p / (s->prm.gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2)};
    HIPCHK(s, launch_freestream(s->stream, s->n, s->nrm, s->kind, Uinf, s->U));
    st = prep_state(s);
    if (st) return st;
    st = sync_and_check(s, "init_freestream");
    s->has_state = (st == QL_OK);
    s->has_eval = s->has_res = false;
    return st;
}

int ql_set_state(ql_solver *s, const double *U, int32_t mem, int32_t project_wall) {
    int st = ensure_ready(s, false);
    if (st) return st;
    if (!U) return fail(s, QL_EINVAL, "U is NULL");
    if (mem != 0 && mem != 1) return fail(s, QL_EINVAL, "mem must be 0 or 1");
    (void)hipSetDevice(s->device);
    const size_t bytes = sizeof(double) * 4 * (size_t)s->n;
    const double *src = U;
    if (mem == 0) {
        HIPCHK(s, hipMemcpyAsync(s->tmp, U, bytes, hipMemcpyHostToDevice, s->stream));
        src = s->tmp;
    }
    HIPCHK(s, launch_permute_state(s->stream, s->n, src, s->dperm, s->nrm, s->kind,
                                   project_wall ? 1 : 0, s->U));
    st = prep_state(s);
    if (st) return st;
    st = sync_and_check(s, "set_state");
    s->has_state = (st == QL_OK);
    s->has_eval = s->has_res = false;
    return st;
}

int ql_fetch_state(ql_solver *s, double *U, int32_t mem) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!U) return fail(s, QL_EINVAL, "U is NULL");
    if (mem != 0 && mem != 1) return fail(s, QL_EINVAL, "mem must be 0 or 1");
    (void)hipSetDevice(s->device);
    double *dst = (mem == 1) ? U : s->tmp;
    HIPCHK(s, launch_unpermute_state(s->stream, s->n, s->U, s->dperm, dst));
    if (mem == 0)
        HIPCHK(s, hipMemcpyAsync(U, s->tmp, sizeof(double) * 4 * (size_t)s->n,
                                 hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QL_OK;
}

int ql_step(ql_solver *s, int32_t n_iter, double *res_hist) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (n_iter < 0) return fail(s, QL_EINVAL, "n_iter < 0");
    if (n_iter == 0) return QL_OK;
    (void)hipSetDevice(s->device);
    if (n_iter > s->reshist_cap) {
        dfree(s->reshist);
        HIPCHK(s, dalloc(&s->reshist, (size_t)4 * n_iter));
        s->reshist_cap = n_iter;
    }
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    st = reset_err(s);
    if (st) return st;
    const int nblk = num_blocks(s->n);
    const double inv_nupd = s->n_upd > 0 ? 1.0 / s->n_upd : 0.0;
    for (int it = 0; it < n_iter; ++it) {
        for (int rk = 1; rk <= 4; ++rk) {
            st = run_gradients(s, c, fp.limiter != 0);
            if (st) return st;
            Timer t(s, 2);
            st = launch_stage(s, c, fp, rk, nullptr, rk == 1 ? s->partial : nullptr);
            if (st) return st;
            t.done();
            s->qcur = 1 - s->qcur;
        }
        Timer t(s, 3);
        HIPCHK(s, launch_resnorm(s->stream, nblk, s->partial, inv_nupd, s->reshist + 4 * it));
        t.done();
    }
    std::vector<double> hist((size_t)4 * n_iter);
    HIPCHK(s, hipMemcpyAsync(hist.data(), s->reshist, sizeof(double) * 4 * n_iter,
                             hipMemcpyDeviceToHost, s->stream));
    st = sync_and_check(s, "step");
    harvest_timing(s);
    s->has_eval = false;
    if (st) return st;
    if (res_hist) std::memcpy(res_hist, hist.data(), sizeof(double) * 4 * n_iter);
    std::memcpy(s->last_res, &hist[(size_t)4 * (n_iter - 1)], sizeof s->last_res);
    s->has_res = true;
    return QL_OK;
}

int ql_residual_norm(const ql_solver *s, double out[4]) {
    if (!s || !out) return QL_EINVAL;
    if (!s->has_res) return QL_ESTATE;
    std::memcpy(out, s->last_res, sizeof s->last_res);
    return QL_OK;
}

int ql_evaluate(ql_solver *s) {
    int st = ensure_ready(s, true);
    if (st) return st;
    (void)hipSetDevice(s->device);
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    st = reset_err(s);
    if (st) return st;
    st = run_gradients(s, c, true);
    if (st) return st;
    st = launch_stage(s, c, fp, 0, s->R, nullptr);
    if (st) return st;
    st = sync_and_check(s, "evaluate");
    harvest_timing(s);
    s->has_eval = (st == QL_OK);
    return st;
}

int ql_debug_fetch(ql_solver *s, int32_t what, double *out) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!out) return fail(s, QL_EINVAL, "out is NULL");
    if (what < 0 || what > 5) return fail(s, QL_EINVAL, "bad inspection index %d", what);
    if ((what == 1 || what == 2 || what == 4 || what == 5) && !s->has_eval)
        return fail(s, QL_ESTATE, "call ql_evaluate first");
    (void)hipSetDevice(s->device);
    const int n = s->n;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    std::vector<double> h;
    auto get = [&](const void *src, size_t count) -> int {
        h.resize(count);
        HIPCHK(s, hipMemcpy(h.data(), src, sizeof(double) * count, hipMemcpyDeviceToHost));
        return QL_OK;
    };
    switch (what) {
    case 0:
        if ((st = get(s->q[s->qcur], (size_t)4 * n))) return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 4; ++r) out[(size_t)r * n + s->perm[q]] = h[(size_t)4 * q + r];
        break;
    case 1:
        if ((st = get(s->g[s->gfin], (size_t)8 * n))) return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 8; ++r) out[(size_t)r * n + s->perm[q]] = h[(size_t)8 * q + r];
        break;
    case 2:
        if ((st = get(s->R, (size_t)4 * n))) return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 4; ++r) out[(size_t)r * n + s->perm[q]] = h[(size_t)r * n + q];
        break;
    case 3:
        if ((st = get(s->dt, (size_t)n))) return st;
        for (int q = 0; q < n; ++q) out[s->perm[q]] = h[q];
        break;
    case 4:
    case 5:
        if ((st = get(s->qmm, (size_t)8 * n))) return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 4; ++r)
                out[(size_t)r * n + s->perm[q]] = h[(size_t)8 * q + (what == 4 ? 0 : 4) + r];
        break;
    }
    return QL_OK;
}

int ql_debug_flags(ql_solver *s, uint8_t *out) {
    int st = ensure_ready(s, false);
    if (st) return st;
    if (!out) return fail(s, QL_EINVAL, "out is NULL");
    (void)hipSetDevice(s->device);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    std::vector<uint8_t> h(s->nnz);
    if (s->nnz) HIPCHK(s, hipMemcpy(h.data(), s->flag, s->nnz, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < s->nnz; ++k) out[s->eperm[k]] = h[k];
    return QL_OK;
}

int ql_forces(ql_solver *s, double *cl, double *cd) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!cl || !cd) return fail(s, QL_EINVAL, "null output");
    if (s->nw < 3) return fail(s, QL_EINVAL, "fewer than 3 wall points");
    (void)hipSetDevice(s->device);
    HIPCHK(s, launch_forces(s->stream, s->nw, s->wall, s->xy, s->nrm, s->U, s->n, s->prm.gamma,
                            1.0 / s->prm.gamma, s->fscratch, s->fout));
    double F[2];
    HIPCHK(s, hipMemcpyAsync(F, s->fout, sizeof F, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const double a = s->prm.alpha_deg * M_PI / 180.0;
    const double qinf = 0.5 * s->prm.mach * s->prm.mach;
    *cl = (-F[0] * std::sin(a) + F[1] * std::cos(a)) / qinf;
    *cd = (F[0] * std::cos(a) + F[1] * std::sin(a)) / qinf;
    return QL_OK;
}

int ql_set_timing(ql_solver *s, int32_t enable) {
    if (!s) return QL_EINVAL;
    s->timing = enable != 0;
    for (int k = 0; k < 4; ++k) {
        s->tsum[k] = 0.0;
        s->tcnt[k] = 0;
    }
    return QL_OK;
}

int ql_kernel_time(const ql_solver *s, int32_t which, double *total_ms, int64_t *count) {
    if (!s || which < 0 || which > 3) return QL_EINVAL;
    if (total_ms) *total_ms = s->tsum[which];
    if (count) *count = s->tcnt[which];
    return QL_OK;
}

}  // extern "C"
