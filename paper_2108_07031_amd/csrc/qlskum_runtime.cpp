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
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/qlskum.h"
#include "qlskum_internal.h"

namespace ql {  // the warm-start network's runtime (qlskum_mlp_runtime.cpp)
hipStream_t mlp_stream(const ql_mlp *m);
int mlp_width(const ql_mlp *m, int end);
bool mlp_ready(const ql_mlp *m);
}  // namespace ql

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

    // cloud (library order); a cloud is one or more independent cases, each a
    // contiguous range of points with its own freestream
    int n = 0;
    int64_t nnz = 0;
    int ncase = 0;
    std::vector<int> case_lo;        // [ncase+1] first point of each case
    std::vector<int> case_nupd;      // updated (interior + wall) points per case
    int outer_bad = -1;  // first outer point (caller order) with a singular split stencil
    std::vector<int> wall_lo;        // [ncase+1] offsets into the wall list
    std::vector<double> case_mach, case_alpha;
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
    float4 *gf[3] = {nullptr, nullptr, nullptr};  // mixed q-derivatives: first pass, iterates
    bool grad_f32 = false;  // the last q-derivatives came from the FP32-data sweeps
    ql_progress_fn progress = nullptr;  // batched-run progress callback
    void *progress_user = nullptr;
    double *lsi = nullptr;
    double *Rpart[2] = {nullptr, nullptr};  // [4][n] partial sums of a split flux sweep
    int *fhalo_ptr = nullptr, *fhalo_idx = nullptr;  // tiles of kFluxTile points
    uint16_t *flidx = nullptr;
    int fmax_slots = 0;
    std::vector<int> fslots;  // image size (records) of every flux tile
    double *reshist = nullptr, *fscratch = nullptr, *fout = nullptr;
    int *case_of = nullptr, *chunk_beg = nullptr, *chunk_ptr = nullptr, *ctr = nullptr;
    int *dwall_lo = nullptr, *wctr = nullptr;  // warm start: wall ranges, residual row counter
    uint8_t *wsel = nullptr;                    // warm start: per-case choice
    double *wres = nullptr;                     // warm start: [2][ncase][4] residual norms
    uint8_t *case_active = nullptr, *tile_active = nullptr;
    // inv_nupd: [2][ncase] 1 / (points in the residual norm): interior and
    // wall points; all points (kinetic outer condition)
    double *uinf = nullptr, *part = nullptr, *inv_nupd = nullptr;
    int nchunk = 0;
    int zero = 0;  // source of the history-row counter reset
    int reshist_cap = 0;
    ErrWord *errw = nullptr;
    ErrWord *errw_outer = nullptr;  // singular split stencils of outer points (set-up)
    ErrWord err_clear = kErrClear;  // source of the error-word reset copies
    // batched runs: per-case error words and the device retirement state
    ErrWord *case_err = nullptr;
    std::vector<ErrWord> case_err_clear;  // [ncase] source of the reset copies
    double *bt_ref = nullptr, *bt_last = nullptr, *bt_drop = nullptr;
    int *bt_iters = nullptr;
    bool retire_on = false;  // iterations enqueued now retire cases on the device
    // precision switch of mixed batched runs: per-case and per-tile flux
    // precision (1 FP32, 0 FP64), the switch threshold and iteration
    uint8_t *case_prec = nullptr, *tile_prec = nullptr;
    double *bt_switch = nullptr;
    int *bt_swit = nullptr;
    bool hybrid = false;  // iterations enqueued now run both flux kernels
    std::vector<int32_t> case_switch;  // per case, of the last ql_batch_run
    // batched runs after retirements: the tiles still holding an active case
    // (device list, its host source and length); the tiled sweeps enqueued
    // while live_on is set launch over the list only
    int *tile_list = nullptr;
    std::vector<int> tile_list_h;
    int ntile_live = 0;
    bool live_on = false;
    // ql_step without a history: the iterations' status and last norms are
    // collected by the next call (rows of history written, and where)
    int step_pending = 0;
    const double *pending_hist = nullptr;
    // ql_step_static: this device's fixed history array, and the flag that
    // keeps the iterations it enqueues free of allocating calls
    double *scratch = nullptr;
    bool no_alloc = false;
    int qcur = 0, gfin = 0;
    std::vector<double> last_res;  // [ncase][4]
    std::vector<int32_t> case_status;  // per case, of the last ql_batch_run
    std::vector<double> uinf_host;  // [ncase][4], source of the s->uinf copy

    // one pseudo-time iteration captured as a graph (batched runs)
    hipGraphExec_t graph = nullptr;
    int graph_qcur = -1;
    bool graph_hybrid = false;  // the captured iteration runs both flux kernels
    int graph_live = 0;  // ... over this many listed tiles (0: every tile)
    bool capturing = false;

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
    dfree(s->g[1]); dfree(s->g[2]); dfree(s->qmm); dfree(s->reshist);
    dfree(s->fscratch); dfree(s->fout); dfree(s->errw); dfree(s->lsi); dfree(s->Rpart[0]);
    dfree(s->Rpart[1]); dfree(s->errw_outer);
    dfree(s->fhalo_ptr); dfree(s->fhalo_idx); dfree(s->flidx);
    dfree(s->q32[0]); dfree(s->q32[1]); dfree(s->g32); dfree(s->qmm32);
    dfree(s->gf[0]); dfree(s->gf[1]); dfree(s->gf[2]);
    dfree(s->case_of); dfree(s->chunk_beg); dfree(s->chunk_ptr); dfree(s->ctr);
    dfree(s->dwall_lo); dfree(s->wctr); dfree(s->wsel); dfree(s->wres);
    dfree(s->case_active); dfree(s->tile_active); dfree(s->tile_list); dfree(s->uinf); dfree(s->part);
    dfree(s->inv_nupd); dfree(s->case_err); dfree(s->bt_ref); dfree(s->bt_last);
    dfree(s->bt_drop); dfree(s->bt_iters); dfree(s->case_prec); dfree(s->tile_prec);
    dfree(s->bt_switch); dfree(s->bt_swit);
    s->case_switch.clear();
    s->step_pending = 0;
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    s->graph_qcur = -1;
    s->fmax_slots = 0;
    s->fslots.clear();
    s->ncase = 0;
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

// Hilbert order of the n points x[0..n), y[0..n) (indices relative to them).
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

// Reverse Cuthill-McKee order of the points lo..hi-1 (one case; indices
// relative to lo) on the neighbour graph: breadth-first from a
// pseudo-peripheral point (George and Liu: restart from the least-connected
// point of the last level while the level count grows), each point's
// unvisited neighbours taken by increasing neighbour count, ties by index;
// every connected part in turn; the whole order reversed.
std::vector<int> rcm_order(int lo, int hi, const int32_t *ptr, const int32_t *idx) {
    const int n = hi - lo;
    auto deg = [&](int p) { return ptr[lo + p + 1] - ptr[lo + p]; };
    std::vector<int> order, level(n, -1), queue, nb;
    order.reserve(n);
    std::vector<char> done(n, 0);
    // levels of a breadth-first search from r (over points not yet ordered);
    // returns the depth and leaves the last level's least-connected point in far
    auto bfs_depth = [&](int r, int &far) {
        queue.assign(1, r);
        level[r] = 0;
        std::vector<int> seen(1, r);
        int depth = 0;
        far = r;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int p = queue[h];
            if (level[p] > depth) {
                depth = level[p];
                far = p;
            } else if (level[p] == depth && deg(p) < deg(far)) {
                far = p;
            }
            for (int k = ptr[lo + p]; k < ptr[lo + p + 1]; ++k) {
                const int i = idx[k] - lo;
                if (level[i] < 0 && !done[i]) {
                    level[i] = level[p] + 1;
                    queue.push_back(i);
                    seen.push_back(i);
                }
            }
        }
        for (int p : seen) level[p] = -1;
        return depth;
    };
    std::vector<int> by_deg(n);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int a, int b) { return deg(a) < deg(b); });
    for (int start : by_deg) {
        if (done[start]) continue;
        int r = start, far = start, depth = bfs_depth(r, far);
        for (int it = 0; it < 8; ++it) {  // pseudo-peripheral start
            int far2 = far;
            const int d2 = bfs_depth(far, far2);
            if (d2 <= depth) break;
            r = far;
            depth = d2;
            far = far2;
        }
        queue.assign(1, r);
        done[r] = 1;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int p = queue[h];
            order.push_back(p);
            nb.clear();
            for (int k = ptr[lo + p]; k < ptr[lo + p + 1]; ++k) {
                const int i = idx[k] - lo;
                if (!done[i]) {
                    done[i] = 1;
                    nb.push_back(i);
                }
            }
            std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) {
                return deg(a) < deg(b) || (deg(a) == deg(b) && a < b);
            });
            queue.insert(queue.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Tiles of T consecutive points: the sorted list of each tile's halo
// (neighbours outside the tile) and every entry's slot in the tile's LDS
// image (own point j -> j, halo point h -> T + h).  Returns the largest image
// (own slots + halo), or INT_MAX when a slot would not fit 16 bits.
int build_tiles(int n, int T, const std::vector<int> &ptr, const std::vector<int> &idx,
                std::vector<int> &hptr, std::vector<int> &hidx, std::vector<uint16_t> &lidx) {
    const int ntile = (n + T - 1) / T;
    hptr.assign(ntile + 1, 0);
    hidx.clear();
    lidx.assign(idx.size(), 0);
    std::vector<int> stamp(n, -1), slot(n, 0), h;
    int max_slots = 0;
    for (int t = 0; t < ntile; ++t) {
        const int base = t * T, end = std::min(n, base + T);
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
        const int slots = T + (int)h.size();
        if (slots > 65535) return INT_MAX;
        for (size_t j = 0; j < h.size(); ++j) slot[h[j]] = T + (int)j;
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
    c.lsi = s->lsi;
    const bool ftiles = s->fhalo_ptr && !s->untiled;
    c.fhalo_ptr = ftiles ? s->fhalo_ptr : nullptr;
    c.fhalo_idx = ftiles ? s->fhalo_idx : nullptr;
    c.flidx = ftiles ? s->flidx : nullptr;
    c.fmax_slots = ftiles ? s->fmax_slots : 0;
    c.case_of = s->case_of;
    c.case_active = s->case_active;
    c.tile_active = s->tile_active;
    c.uinf = s->uinf;
    c.case_err = s->case_err;
    c.tile_prec = s->hybrid ? s->tile_prec : nullptr;
    c.tile_list = s->live_on ? s->tile_list : nullptr;
    c.ntile_live = s->live_on ? s->ntile_live : 0;
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
    f.order = s->prm.order;
    f.kobc = s->prm.outer_bc;
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
    if (p->reorder < 0 || p->reorder > 2) return fail(s, QL_EINVAL, "reorder must be 0, 1 or 2");
    if (p->flux_lds < 0 || p->flux_lds > 160 * 1024)
        return fail(s, QL_EINVAL, "flux_lds must lie in [0, 163840] bytes");
    if (p->grad_lds < 0 || p->grad_lds > 160 * 1024)
        return fail(s, QL_EINVAL, "grad_lds must lie in [0, 163840] bytes");
    if (p->order != 1 && p->order != 2) return fail(s, QL_EINVAL, "order must be 1 or 2");
    if (p->flux_split < 0 || p->flux_split > 2)
        return fail(s, QL_EINVAL, "flux_split must be 0, 1 or 2");
    if (p->outer_bc != 0 && p->outer_bc != 1) return fail(s, QL_EINVAL, "outer_bc must be 0 or 1");
    if (p->mixed_grad != 0 && p->mixed_grad != 1)
        return fail(s, QL_EINVAL, "mixed_grad must be 0 or 1");
    if (!(p->mixed_switch >= 0.0 && p->mixed_switch < 1.0))
        return fail(s, QL_EINVAL, "mixed_switch must lie in [0, 1)");
    if (p->outer_bc == 1 && s->has_cloud && s->outer_bad >= 0)
        return fail(s, QL_ESINGULAR,
                    "kinetic outer condition: singular split stencil at outer point %d",
                    s->outer_bad);
    return QL_OK;
}

int reset_err(ql_solver *s) {
    HIPCHK(s, hipMemcpyAsync(s->errw, &s->err_clear, sizeof(ErrWord), hipMemcpyHostToDevice,
                             s->stream));
    return QL_OK;
}

int reset_case_err(ql_solver *s) {
    HIPCHK(s, hipMemcpyAsync(s->case_err, s->case_err_clear.data(), sizeof(ErrWord) * s->ncase,
                             hipMemcpyHostToDevice, s->stream));
    return QL_OK;
}

// Status of a device error word (library-order point and code).
static int err_status(ql_solver *s, ErrWord w, const char *what) {
    const int code = err_code(w), pt = err_point(w);
    if (code == kErrNone) return QL_OK;
    const int up = (pt >= 0 && pt < s->n) ? s->perm[pt] : -1;
    switch (code) {
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

// Synchronise and read the device error word.
static int read_err(ql_solver *s, ErrWord *w) {
    HIPCHK(s, hipMemcpyAsync(w, s->errw, sizeof(ErrWord), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QL_OK;
}

// Synchronise and turn the device error word into a status.
int sync_and_check(ql_solver *s, const char *what) {
    ErrWord w = kErrClear;
    int st = read_err(s, &w);
    if (st) return st;
    return err_status(s, w, what);
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
        if (s->timing && !s->capturing && !s->no_alloc) {
            a = take_event(s);
            if (a) (void)hipEventRecord(a, s->stream);
        }
    }
    void done() {
        if (s->timing && !s->capturing && !s->no_alloc && a) {
            hipEvent_t b = take_event(s);
            if (b) (void)hipEventRecord(b, s->stream);
            s->pending.push_back({kind, a, b});
        }
    }
};

// One stage's q-derivatives: first pass + n_inner Jacobi iterations.
// Mixed precision with FP32 data (mixed_grad 0, no precision switch): the
// sweeps that gather FP32 copies, the first pass into gf[0] (or g32 with no
// inner iteration), the iterates alternating between gf[1] and gf[2], the
// last into g32.  Otherwise the FP64 sweeps: the first pass goes to g[2]
// when inner iterations follow (they read it as g0), the iterates alternate
// between g[0] and g[1], the final one is g[gfin]; in mixed precision they
// also write the FP32 copies the mixed flux sweep reads, and skip the FP64
// bounds and final iterate that only inspection (fp64_out) or a run that
// switches cases to FP64 fluxes reads.
int run_gradients(ql_solver *s, const DevCloud &c, bool want_bounds, bool fp64_out) {
    const bool mixed = s->prm.precision == 1;
    s->grad_f32 = mixed && !s->hybrid && s->prm.mixed_grad == 0;
    if (s->grad_f32) {
        const int ni = s->prm.n_inner;
        {
            Timer t(s, 0);
            HIPCHK(s, launch_grad0_f(s->stream, c, s->prm.grad_lds, s->q32[s->qcur],
                                     ni > 0 ? s->gf[0] : s->g32, s->qmm32, want_bounds ? 1 : 0));
            t.done();
        }
        const float4 *cur = s->gf[0];
        for (int k = 0; k < ni; ++k) {
            float4 *nxt = (k == ni - 1) ? s->g32 : s->gf[1 + (k & 1)];
            Timer t(s, 1);
            HIPCHK(s, launch_gradk_f(s->stream, c, s->prm.grad_lds, s->gf[0], cur, nxt));
            t.done();
            cur = nxt;
        }
        return QL_OK;
    }
    const int first = s->prm.n_inner > 0 ? 2 : 0;
    const bool skip64 = mixed && !fp64_out && !s->hybrid;
    Shadow sh{nullptr, nullptr, nullptr};
    if (mixed) {
        sh.qmm32 = s->qmm32;
        if (s->prm.n_inner == 0) sh.g32 = s->g32;
    }
    {
        Timer t(s, 0);
        HIPCHK(s, launch_grad0(s->stream, c, s->prm.grad_lds, s->q[s->qcur], s->g[first],
                               skip64 ? nullptr : s->qmm, want_bounds ? 1 : 0, sh));
        t.done();
    }
    int cur = first;
    for (int k = 0; k < s->prm.n_inner; ++k) {
        const int nxt = (cur == 0) ? 1 : 0;
        const bool last = k == s->prm.n_inner - 1;
        float4 *g32 = (mixed && last) ? s->g32 : nullptr;
        Timer t(s, 1);
        HIPCHK(s, launch_gradk(s->stream, c, s->prm.grad_lds, s->g[2], s->g[cur],
                               (skip64 && last) ? nullptr : s->g[nxt], g32));
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

// LDS bytes a flux workgroup may stage its tile image in.  The defaults keep
// the workgroups that the kernels' register use allows per CU resident
// (3 for FP64 with the limiter, 4 otherwise; 160 KB of LDS per CU).
int flux_lds_budget(const ql_solver *s) {
    if (s->prm.flux_lds > 0) return s->prm.flux_lds;
    return (s->prm.precision == 0 && s->prm.limiter) ? 52 * 1024 : 40 * 1024;
}

// One flux-residual launch (stage 0: evaluate into R; 1..4: RK stage).
int launch_stage(ql_solver *s, const DevCloud &c, const FlowParams &fp, int stage, double *Rout) {
    const int a = s->qcur, b = 1 - s->qcur;
    const int lds = flux_lds_budget(s);
    if (s->hybrid) {
        // each kernel takes the tiles of its precision (tile_prec); the FP64
        // one with its own default LDS budget
        ql_params saved = s->prm;
        s->prm.precision = 0;
        const int lds64 = flux_lds_budget(s);
        s->prm = saved;
        HIPCHK(s, launch_flux(s->stream, c, fp, stage, lds64, s->q[a], s->g[s->gfin], s->qmm, s->U,
                              s->Un, s->dt, s->q[b], Rout, s->q32[b], s->errw, 0, s->Rpart));
        HIPCHK(s, launch_flux_mixed(s->stream, c, fp, stage, lds, s->q[a], s->q32[a], s->g32,
                                    s->qmm32, s->U, s->Un, s->dt, s->q[b], s->q32[b], Rout,
                                    s->errw));
        return QL_OK;
    }
    if (s->prm.precision == 1)
        HIPCHK(s, launch_flux_mixed(s->stream, c, fp, stage, lds, s->q[a], s->q32[a], s->g32,
                                    s->qmm32, s->U, s->Un, s->dt, s->q[b], s->q32[b], Rout,
                                    s->errw));
    else
        HIPCHK(s, launch_flux(s->stream, c, fp, stage, lds, s->q[a], s->g[s->gfin], s->qmm, s->U,
                              s->Un, s->dt, s->q[b], Rout, s->q32[b], s->errw,
                              fp.order == 2 ? 2 * s->prm.flux_split : 0, s->Rpart));
    return QL_OK;
}

// Enqueue one pseudo-time iteration: four stages, then the residual norms of
// stage 1 into history row *ctr.
int enqueue_iteration(ql_solver *s, const DevCloud &c, const FlowParams &fp, int hist_cap,
                      double *hist) {
    for (int rk = 1; rk <= 4; ++rk) {
        int st = QL_OK;
        // the first-order scheme needs no q-derivatives
        if (fp.order == 2 && (st = run_gradients(s, c, fp.limiter != 0, false))) return st;
        Timer t(s, 2);
        st = launch_stage(s, c, fp, rk, rk == 1 ? s->R : nullptr);
        if (st) return st;
        t.done();
        s->qcur = 1 - s->qcur;
    }
    Timer t(s, 3);
    const Retire rt{s->retire_on ? 1 : 0, s->bt_drop, s->bt_ref, s->bt_iters, s->bt_last,
                    s->case_active, s->case_err, s->bt_switch,
                    s->hybrid ? s->case_prec : nullptr, s->bt_swit};
    HIPCHK(s, launch_resnorm(s->stream, s->R, s->n, s->nchunk, s->chunk_beg, s->part, s->ncase,
                             s->chunk_ptr, s->inv_nupd + (fp.kobc ? s->ncase : 0), s->ctr,
                             hist_cap, hist, rt, s->case_of, s->tile_active, s->tile_prec));
    t.done();
    return QL_OK;
}

int ensure_history(ql_solver *s, int rows) {
    const int need = rows * s->ncase;
    if (need > s->reshist_cap) {
        dfree(s->reshist);
        HIPCHK(s, dalloc(&s->reshist, (size_t)4 * need));
        s->reshist_cap = need;
        if (s->graph) (void)hipGraphExecDestroy(s->graph);  // the graph holds the old buffer
        s->graph = nullptr;
    }
    return QL_OK;
}

int reset_counter(ql_solver *s) {
    HIPCHK(s, hipMemcpyAsync(s->ctr, &s->zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    return QL_OK;
}

// Capture one iteration into s->graph (rows of history: capacity per replay
// block is reshist_cap / ncase).
int capture_iteration(ql_solver *s) {
    if (s->graph && s->graph_qcur == s->qcur && s->graph_hybrid == s->hybrid &&
        s->graph_live == (s->live_on ? s->ntile_live : 0))
        return QL_OK;
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    const int q0 = s->qcur;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    s->capturing = true;
    int st = enqueue_iteration(s, c, fp, s->reshist_cap / s->ncase, s->reshist);
    s->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(s, QL_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess)
        return fail(s, QL_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e2));
    s->qcur = q0;  // capture enqueued nothing; the four stage flips cancel anyway
    s->graph_qcur = q0;
    s->graph_hybrid = s->hybrid;
    s->graph_live = s->live_on ? s->ntile_live : 0;
    return QL_OK;
}

void drop_graph(ql_solver *s) {
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    s->graph_qcur = -1;
}

// Address of this library's fixed history array on `device` (looked up once
// per device, with the device current; each GPU holds its own copy).
hipError_t scratch_of_device(int device, double **ptr) {
    static std::mutex mu;
    static std::vector<double *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
    if (!addr[device]) {
        const hipError_t e = scratch_address(&addr[device]);
        if (e != hipSuccess) return e;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// Collect the outcome of iterations that ql_step enqueued without a
// history: their last residual norms and the error word (one
// synchronisation).  A failure is returned to the call that collects it.
int settle(ql_solver *s) {
    if (!s->step_pending) return QL_OK;
    const size_t row = (size_t)s->step_pending - 1;
    s->step_pending = 0;
    (void)hipSetDevice(s->device);
    HIPCHK(s, hipMemcpyAsync(s->last_res.data(), s->pending_hist + row * s->ncase * 4,
                             sizeof(double) * 4 * s->ncase, hipMemcpyDeviceToHost, s->stream));
    const int st = sync_and_check(s, "step");
    harvest_timing(s);
    if (st) return st;
    s->has_res = true;
    return QL_OK;
}

int ensure_ready(ql_solver *s, bool need_state) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    if (int st = settle(s)) return st;
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
    p->flux_lds = 0;
    p->grad_lds = 0;
    p->order = 2;
    p->flux_split = 0;
    p->outer_bc = 0;
    p->mixed_grad = 0;
    p->mixed_switch = 0.0;
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
    if (scratch_of_device(device, &s->scratch) != hipSuccess) {
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

static int upload_freestream(ql_solver *s);

int ql_set_params(ql_solver *s, const ql_params *p) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    int st = check_params(s, p);
    if (st) return st;
    s->prm = *p;
    drop_graph(s);
    for (int k = 0; k < 2; ++k)
        if (s->has_cloud && p->flux_split && !s->Rpart[k])
            HIPCHK(s, dalloc(&s->Rpart[k], (size_t)4 * s->n));
    if (s->has_cloud) {
        (void)hipSetDevice(s->device);
        return upload_freestream(s);
    }
    return QL_OK;
}

static int upload_freestream(ql_solver *s);

static int upload_impl(ql_solver *s, int32_t ncase, const int64_t *case_ptr, int64_t n64,
                       const double *x, const double *y, const double *nx, const double *ny,
                       const uint8_t *kind, const int32_t *nbr_ptr, const int32_t *nbr_idx,
                       const uint8_t *nbr_flag, const double *mach, const double *alpha) {
    if (!s) return QL_EINVAL;
    if (s->poisoned) return QL_EDEVICE;
    if (!x || !y || !nx || !ny || !kind || !nbr_ptr || (!nbr_idx && n64 > 0))
        return fail(s, QL_EINVAL, "null array argument");
    if (n64 < 1 || n64 > INT_MAX / 8) return fail(s, QL_EINVAL, "n = %lld out of range", (long long)n64);
    const int n = (int)n64;
    if (ncase < 1 || ncase > n) return fail(s, QL_EINVAL, "ncase = %d out of range", ncase);
    if (case_ptr[0] != 0 || case_ptr[ncase] != n64)
        return fail(s, QL_EINVAL, "case_ptr must start at 0 and end at n");
    for (int c = 0; c < ncase; ++c)
        if (case_ptr[c + 1] <= case_ptr[c]) return fail(s, QL_EINVAL, "case %d is empty", c);
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
    for (int c = 0; c < ncase; ++c) {
        const int lo = (int)case_ptr[c], hi = (int)case_ptr[c + 1];
        for (int p = lo; p < hi; ++p)
            for (int k = nbr_ptr[p]; k < nbr_ptr[p + 1]; ++k) {
                const int i = nbr_idx[k];
                if (i < lo || i >= hi || i == p)
                    return fail(s, QL_EINVAL,
                                "neighbour entry %d of point %d is out of its case's range or self",
                                k, p);
                if (nbr_flag && (nbr_flag[k] & ~0x0f))
                    return fail(s, QL_EINVAL, "bad split flag at entry %d", k);
            }
        if (mach && (!(mach[c] >= 0.0) || !std::isfinite(mach[c])))
            return fail(s, QL_EINVAL, "bad Mach number of case %d", c);
        if (alpha && !std::isfinite(alpha[c])) return fail(s, QL_EINVAL, "bad alpha of case %d", c);
    }
    (void)hipSetDevice(s->device);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    free_cloud(s);

    // point order: each case keeps its range; Hilbert order inside it
    std::vector<int> perm(n);
    for (int c = 0; c < ncase; ++c) {
        const int lo = (int)case_ptr[c], hi = (int)case_ptr[c + 1];
        if (s->prm.reorder == 1) {
            const std::vector<int> o = hilbert_order(hi - lo, x + lo, y + lo);
            for (int j = 0; j < hi - lo; ++j) perm[lo + j] = lo + o[j];
        } else if (s->prm.reorder == 2) {
            const std::vector<int> o = rcm_order(lo, hi, nbr_ptr, nbr_idx);
            for (int j = 0; j < hi - lo; ++j) perm[lo + j] = lo + o[j];
        } else {
            for (int j = lo; j < hi; ++j) perm[j] = j;
        }
    }
    std::vector<int> inv(n);
    for (int q = 0; q < n; ++q) inv[perm[q]] = q;

    // reordered host arrays
    std::vector<double2> hxy(n), hnrm(n);
    std::vector<uint8_t> hkind(n), hflag(nbr_flag ? nnz : 0);
    std::vector<int> hptr(n + 1), hidx(nnz), hcase(n);
    std::vector<int64_t> eperm(nnz);
    hptr[0] = 0;
    for (int c = 0; c < ncase; ++c)
        for (int q = (int)case_ptr[c]; q < (int)case_ptr[c + 1]; ++q) hcase[q] = c;
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
    // per case: walls in the caller's order, updated-point counts, chunks of
    // the residual reduction (never straddling a case)
    constexpr int kChunk = 4096;
    std::vector<int> hwall, wall_lo(ncase + 1, 0), nupd(ncase, 0), cbeg, cptr(ncase + 1, 0);
    std::vector<double> inv_nupd(2 * (size_t)ncase);
    for (int c = 0; c < ncase; ++c) {
        const int lo = (int)case_ptr[c], hi = (int)case_ptr[c + 1];
        for (int p = lo; p < hi; ++p) {
            if (kind[p] == QL_KIND_WALL) hwall.push_back(inv[p]);
            if (kind[p] != QL_KIND_OUTER) ++nupd[c];
        }
        wall_lo[c + 1] = (int)hwall.size();
        inv_nupd[c] = nupd[c] > 0 ? 1.0 / nupd[c] : 0.0;
        inv_nupd[ncase + c] = 1.0 / (hi - lo);
        for (int b = lo; b < hi; b += kChunk) cbeg.push_back(b);
        cptr[c + 1] = (int)cbeg.size();
    }
    const int nchunk = (int)cbeg.size();
    cbeg.push_back(n);
    const int ntile = num_flux_tiles(n);

    s->n = n;
    s->nnz = nnz;
    s->ncase = ncase;
    s->case_lo.assign(case_ptr, case_ptr + ncase + 1);
    s->case_nupd = nupd;
    s->wall_lo = wall_lo;
    s->case_mach.assign(ncase, s->prm.mach);
    s->case_alpha.assign(ncase, s->prm.alpha_deg);
    if (mach) s->case_mach.assign(mach, mach + ncase);
    if (alpha) s->case_alpha.assign(alpha, alpha + ncase);
    s->last_res.assign((size_t)4 * ncase, 0.0);
    s->case_status.assign(ncase, QL_OK);
    s->nw = (int)hwall.size();
    s->nchunk = nchunk;
    HIPCHK(s, dalloc(&s->xy, n)); HIPCHK(s, dalloc(&s->nrm, n)); HIPCHK(s, dalloc(&s->kind, n));
    HIPCHK(s, dalloc(&s->flag, nnz)); HIPCHK(s, dalloc(&s->ptr, n + 1)); HIPCHK(s, dalloc(&s->idx, nnz));
    HIPCHK(s, dalloc(&s->dperm, n)); HIPCHK(s, dalloc(&s->wall, hwall.size()));
    HIPCHK(s, dalloc(&s->lsw, (size_t)8 * n)); HIPCHK(s, dalloc(&s->dmin, n));
    HIPCHK(s, dalloc(&s->lsi, (size_t)3 * n));
    for (int k = 0; k < 2 && s->prm.flux_split; ++k) HIPCHK(s, dalloc(&s->Rpart[k], (size_t)4 * n));
    HIPCHK(s, dalloc(&s->U, (size_t)4 * n)); HIPCHK(s, dalloc(&s->Un, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->dt, n)); HIPCHK(s, dalloc(&s->R, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->tmp, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->q[0], (size_t)2 * n)); HIPCHK(s, dalloc(&s->q[1], (size_t)2 * n));
    HIPCHK(s, dalloc(&s->g[0], (size_t)4 * n)); HIPCHK(s, dalloc(&s->g[1], (size_t)4 * n));
    HIPCHK(s, dalloc(&s->g[2], (size_t)4 * n));
    HIPCHK(s, dalloc(&s->qmm, (size_t)4 * n));
    HIPCHK(s, dalloc(&s->q32[0], n)); HIPCHK(s, dalloc(&s->q32[1], n));
    HIPCHK(s, dalloc(&s->g32, (size_t)2 * n)); HIPCHK(s, dalloc(&s->qmm32, (size_t)2 * n));
    for (int k = 0; k < 3; ++k) HIPCHK(s, dalloc(&s->gf[k], (size_t)2 * n));
    HIPCHK(s, dalloc(&s->fscratch, (size_t)3 * std::max<size_t>(hwall.size(), 1)));
    HIPCHK(s, dalloc(&s->fout, 2)); HIPCHK(s, dalloc(&s->errw, 1));
    HIPCHK(s, dalloc(&s->errw_outer, 1)); HIPCHK(s, dalloc(&s->case_err, ncase));
    HIPCHK(s, dalloc(&s->bt_ref, ncase)); HIPCHK(s, dalloc(&s->bt_last, (size_t)4 * ncase));
    HIPCHK(s, dalloc(&s->bt_drop, 1)); HIPCHK(s, dalloc(&s->bt_iters, ncase));
    HIPCHK(s, dalloc(&s->case_prec, ncase)); HIPCHK(s, dalloc(&s->tile_prec, ntile));
    HIPCHK(s, dalloc(&s->bt_switch, 1)); HIPCHK(s, dalloc(&s->bt_swit, ncase));
    s->case_err_clear.assign(ncase, kErrClear);
    HIPCHK(s, dalloc(&s->case_of, n)); HIPCHK(s, dalloc(&s->uinf, (size_t)4 * ncase));
    HIPCHK(s, dalloc(&s->case_active, ncase)); HIPCHK(s, dalloc(&s->tile_active, ntile));
    HIPCHK(s, dalloc(&s->tile_list, ntile));
    HIPCHK(s, dalloc(&s->chunk_beg, nchunk + 1)); HIPCHK(s, dalloc(&s->chunk_ptr, ncase + 1));
    HIPCHK(s, dalloc(&s->part, (size_t)4 * nchunk)); HIPCHK(s, dalloc(&s->inv_nupd, 2 * ncase));
    HIPCHK(s, dalloc(&s->ctr, 1));
    HIPCHK(s, dalloc(&s->dwall_lo, ncase + 1)); HIPCHK(s, dalloc(&s->wctr, 1));
    HIPCHK(s, dalloc(&s->wsel, ncase)); HIPCHK(s, dalloc(&s->wres, (size_t)8 * ncase));

    hipStream_t st = s->stream;
    const std::vector<uint8_t> ones_c(ncase, 1), ones_t(ntile, 1);
    HIPCHK(s, hipMemcpyAsync(s->xy, hxy.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->nrm, hnrm.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->kind, hkind.data(), n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->ptr, hptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
    if (nnz) HIPCHK(s, hipMemcpyAsync(s->idx, hidx.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, st));
    if (nbr_flag && nnz) HIPCHK(s, hipMemcpyAsync(s->flag, hflag.data(), nnz, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->dperm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    if (!hwall.empty())
        HIPCHK(s, hipMemcpyAsync(s->wall, hwall.data(), sizeof(int) * hwall.size(), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->case_of, hcase.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->dwall_lo, wall_lo.data(), sizeof(int) * (ncase + 1),
                             hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->case_active, ones_c.data(), ncase, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->tile_active, ones_t.data(), ntile, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->chunk_beg, cbeg.data(), sizeof(int) * (nchunk + 1), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->chunk_ptr, cptr.data(), sizeof(int) * (ncase + 1), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->inv_nupd, inv_nupd.data(), sizeof(double) * inv_nupd.size(),
                             hipMemcpyHostToDevice, st));
    {
        std::vector<int> thptr, thidx;
        std::vector<uint16_t> tlidx;
        const int ms = build_tiles(n, kFluxTile, hptr, hidx, thptr, thidx, tlidx);
        if (ms != INT_MAX) {  // else every flux tile reads from memory
            s->fmax_slots = ms;
            s->fslots.resize(thptr.size() - 1);
            for (size_t t = 0; t + 1 < thptr.size(); ++t)
                s->fslots[t] = kFluxTile + thptr[t + 1] - thptr[t];
            HIPCHK(s, dalloc(&s->fhalo_ptr, thptr.size()));
            HIPCHK(s, dalloc(&s->fhalo_idx, thidx.size()));
            HIPCHK(s, dalloc(&s->flidx, tlidx.size()));
            HIPCHK(s, hipMemcpy(s->fhalo_ptr, thptr.data(), sizeof(int) * thptr.size(),
                                hipMemcpyHostToDevice));
            if (!thidx.empty())
                HIPCHK(s, hipMemcpy(s->fhalo_idx, thidx.data(), sizeof(int) * thidx.size(),
                                    hipMemcpyHostToDevice));
            if (!tlidx.empty())
                HIPCHK(s, hipMemcpy(s->flidx, tlidx.data(), sizeof(uint16_t) * tlidx.size(),
                                    hipMemcpyHostToDevice));
        }
    }
    s->perm.swap(perm);
    s->inv.swap(inv);
    s->eperm.swap(eperm);

    int rc = reset_err(s);
    if (!rc) rc = reset_case_err(s);
    if (rc) return rc;
    HIPCHK(s, hipMemcpyAsync(s->errw_outer, &s->err_clear, sizeof(ErrWord),
                             hipMemcpyHostToDevice, st));
    HIPCHK(s, launch_setup(st, n, s->xy, s->nrm, s->kind, s->ptr, s->idx, s->flag,
                           nbr_flag ? 0 : 1, s->lsw, s->lsi, s->dmin, s->errw, s->errw_outer));
    ErrWord eo = kErrClear;
    HIPCHK(s, hipMemcpyAsync(&eo, s->errw_outer, sizeof eo, hipMemcpyDeviceToHost, st));
    // host buffers above must outlive the asynchronous copies
    rc = sync_and_check(s, "upload");
    const int eop = err_point(eo);
    s->outer_bad = (err_code(eo) != kErrNone && eop >= 0 && eop < n) ? s->perm[eop] : -1;
    if (!rc && s->prm.outer_bc == 1 && s->outer_bad >= 0)
        rc = fail(s, QL_ESINGULAR,
                  "upload: kinetic outer condition: singular split stencil at outer point %d",
                  s->outer_bad);
    if (!rc) rc = upload_freestream(s);
    if (rc) {
        const std::string msg = s->err;
        free_cloud(s);
        s->err = msg;
        return rc;
    }
    s->has_cloud = true;
    return QL_OK;
}

int ql_upload_cloud(ql_solver *s, int64_t n64, const double *x, const double *y,
                    const double *nx, const double *ny, const uint8_t *kind,
                    const int32_t *nbr_ptr, const int32_t *nbr_idx, const uint8_t *nbr_flag) {
    const int64_t cp[2] = {0, n64};
    return upload_impl(s, 1, cp, n64, x, y, nx, ny, kind, nbr_ptr, nbr_idx, nbr_flag, nullptr,
                       nullptr);
}

int ql_batch_upload(ql_solver *s, int32_t ncase, const int64_t *case_ptr, int64_t n,
                    const double *x, const double *y, const double *nx, const double *ny,
                    const uint8_t *kind, const int32_t *nbr_ptr, const int32_t *nbr_idx,
                    const double *mach, const double *alpha_deg) {
    if (!s) return QL_EINVAL;
    if (!case_ptr || !mach || !alpha_deg) return fail(s, QL_EINVAL, "null case array");
    return upload_impl(s, ncase, case_ptr, n, x, y, nx, ny, kind, nbr_ptr, nbr_idx, nullptr, mach,
                       alpha_deg);
}

int ql_cloud_size(const ql_solver *s, int64_t *n, int64_t *nnz) {
    if (!s || !s->has_cloud) return QL_ESTATE;
    if (n) *n = s->n;
    if (nnz) *nnz = s->nnz;
    return QL_OK;
}

// Conserved freestream of every case into s->uinf (rho = 1, p = 1/gamma).
// Conserved freestream of every case into s->uinf (the one-case form takes
// the Mach number and incidence of ql_set_params).  The kinetic outer
// condition reads it at every flux evaluation, whatever set the state.
static int upload_freestream(ql_solver *s) {
    if (s->ncase == 1) {
        s->case_mach[0] = s->prm.mach;
        s->case_alpha[0] = s->prm.alpha_deg;
    }
    s->uinf_host.assign((size_t)4 * s->ncase, 0.0);
    for (int c = 0; c < s->ncase; ++c) {
        const double a = s->case_alpha[c] * M_PI / 180.0;
        const double rho = 1.0, u1 = s->case_mach[c] * std::cos(a), u2 = s->case_mach[c] * std::sin(a);
        const double p = 1.0 / s->prm.gamma;
        double *u = &s->uinf_host[4 * c];
        u[0] = rho;
        u[1] = rho * u1;
        u[2] = rho * u2;
        u[3] = p / (s->prm.gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2);
    }
    HIPCHK(s, hipMemcpyAsync(s->uinf, s->uinf_host.data(), sizeof(double) * s->uinf_host.size(),
                             hipMemcpyHostToDevice, s->stream));
    // the host copy is rewritten by the next call: let this one complete
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QL_OK;
}

int ql_init_freestream(ql_solver *s) {
    int st = ensure_ready(s, false);
    if (st) return st;
    (void)hipSetDevice(s->device);
    if ((st = upload_freestream(s))) return st;
    HIPCHK(s, launch_freestream(s->stream, s->n, s->nrm, s->kind, s->case_of, s->uinf, s->U));
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
    if ((st = ensure_history(s, n_iter))) return st;
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    if ((st = reset_err(s))) return st;
    if ((st = reset_counter(s))) return st;
    for (int it = 0; it < n_iter; ++it)
        if ((st = enqueue_iteration(s, c, fp, s->reshist_cap / s->ncase, s->reshist))) return st;
    s->has_eval = false;
    if (!res_hist) {  // no synchronisation: the next call collects the outcome
        s->step_pending = n_iter;
        s->pending_hist = s->reshist;
        s->has_res = false;
        return QL_OK;
    }
    const size_t rows = (size_t)n_iter * s->ncase * 4;
    std::vector<double> hist(rows);
    HIPCHK(s, hipMemcpyAsync(hist.data(), s->reshist, sizeof(double) * rows, hipMemcpyDeviceToHost,
                             s->stream));
    st = sync_and_check(s, "step");
    harvest_timing(s);
    s->has_eval = false;
    if (st) return st;
    if (res_hist) std::memcpy(res_hist, hist.data(), sizeof(double) * rows);
    std::memcpy(s->last_res.data(), &hist[rows - (size_t)4 * s->ncase],
                sizeof(double) * 4 * s->ncase);
    s->has_res = true;
    return QL_OK;
}

int ql_step_static(ql_solver *s, int32_t n_iter, double *res_hist) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (n_iter < 0) return fail(s, QL_EINVAL, "n_iter < 0");
    if (n_iter == 0) return QL_OK;
    const int cap = kScratchDoubles / (4 * s->ncase);
    if (n_iter > cap)
        return fail(s, QL_EINVAL, "ql_step_static: n_iter = %d exceeds %d rows of %d case(s)",
                    n_iter, cap, s->ncase);
    (void)hipSetDevice(s->device);
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    if ((st = reset_err(s)) || (st = reset_counter(s))) return st;
    // the same iterations as ql_step, with no timing events and the history
    // rows in this device's fixed array
    s->no_alloc = true;
    for (int it = 0; it < n_iter && !st; ++it) st = enqueue_iteration(s, c, fp, cap, s->scratch);
    s->no_alloc = false;
    if (st) return st;
    s->has_eval = false;
    const size_t rows = (size_t)n_iter * s->ncase * 4;
    if (!res_hist) {
        s->step_pending = n_iter;
        s->pending_hist = s->scratch;
        s->has_res = false;
        return QL_OK;
    }
    HIPCHK(s, hipMemcpyAsync(res_hist, s->scratch, sizeof(double) * rows, hipMemcpyDeviceToHost,
                             s->stream));
    if ((st = sync_and_check(s, "step_static"))) return st;
    std::memcpy(s->last_res.data(), res_hist + rows - (size_t)4 * s->ncase,
                sizeof(double) * 4 * s->ncase);
    s->has_res = true;
    return QL_OK;
}

int ql_residual_norm(const ql_solver *s, double out[4]) {
    if (!s || !out) return QL_EINVAL;
    // collecting a pending step's norms changes no observable state but the
    // cached norms themselves
    if (int st = settle(const_cast<ql_solver *>(s))) return st;
    if (!s->has_res) return QL_ESTATE;
    std::memcpy(out, s->last_res.data(), sizeof(double) * 4);
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
    st = run_gradients(s, c, true, true);
    if (st) return st;
    st = launch_stage(s, c, fp, 0, s->R);
    if (st) return st;
    st = sync_and_check(s, "evaluate");
    harvest_timing(s);
    s->has_eval = (st == QL_OK);
    return st;
}

int ql_flux_tiles(const ql_solver *s, int32_t *ntile, int32_t *slots) {
    if (!s || !ntile) return QL_EINVAL;
    if (!s->has_cloud) return QL_ESTATE;
    *ntile = (int32_t)s->fslots.size();
    if (slots)
        for (size_t t = 0; t < s->fslots.size(); ++t) slots[t] = s->fslots[t];
    return QL_OK;
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
    // FP32 arrays (the mixed q-derivatives and bounds), widened
    std::vector<float> hf;
    auto getf = [&](const void *src, size_t count) -> int {
        hf.resize(count);
        HIPCHK(s, hipMemcpy(hf.data(), src, sizeof(float) * count, hipMemcpyDeviceToHost));
        h.assign(hf.begin(), hf.end());
        return QL_OK;
    };
    switch (what) {
    case 0:
        if ((st = get(s->q[s->qcur], (size_t)4 * n))) return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 4; ++r) out[(size_t)r * n + s->perm[q]] = h[(size_t)4 * q + r];
        break;
    case 1:
        if ((st = s->grad_f32 ? getf(s->g32, (size_t)8 * n) : get(s->g[s->gfin], (size_t)8 * n)))
            return st;
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
    case 5: {
        // the bounds are held as offsets from q: q + (qmax - q), within an ulp
        // of qmax (mixed: offsets from the FP32 copy of q, both in FP32)
        if ((st = s->grad_f32 ? getf(s->q32[s->qcur], (size_t)4 * n)
                              : get(s->q[s->qcur], (size_t)4 * n)))
            return st;
        const std::vector<double> hq = h;
        if ((st = s->grad_f32 ? getf(s->qmm32, (size_t)8 * n) : get(s->qmm, (size_t)8 * n)))
            return st;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < 4; ++r)
                out[(size_t)r * n + s->perm[q]] =
                    hq[(size_t)4 * q + r] + h[(size_t)8 * q + (what == 4 ? 0 : 4) + r];
        break;
    }
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

static int case_forces(ql_solver *s, int c, double *cl, double *cd) {
    const int w0 = s->wall_lo[c], nw = s->wall_lo[c + 1] - w0;
    if (nw < 3) return fail(s, QL_EINVAL, "case %d has fewer than 3 wall points", c);
    HIPCHK(s, launch_forces(s->stream, nw, s->wall + w0, s->xy, s->nrm, s->U, s->n, s->prm.gamma,
                            1.0 / s->prm.gamma, s->fscratch, s->fout));
    double F[2];
    HIPCHK(s, hipMemcpyAsync(F, s->fout, sizeof F, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const double mach = (s->ncase == 1) ? s->prm.mach : s->case_mach[c];
    const double alpha = (s->ncase == 1) ? s->prm.alpha_deg : s->case_alpha[c];
    const double a = alpha * M_PI / 180.0;
    const double qinf = 0.5 * mach * mach;
    *cl = (-F[0] * std::sin(a) + F[1] * std::cos(a)) / qinf;
    *cd = (F[0] * std::cos(a) + F[1] * std::sin(a)) / qinf;
    return QL_OK;
}

int ql_forces(ql_solver *s, double *cl, double *cd) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!cl || !cd) return fail(s, QL_EINVAL, "null output");
    (void)hipSetDevice(s->device);
    return case_forces(s, 0, cl, cd);
}

// --- warm start -------------------------------------------------------------

// Stage-1 residual norms of the current U into row *wctr of s->wres, with
// the error word left for the caller to read.
static int warm_eval(ql_solver *s, const DevCloud &c, const FlowParams &fp) {
    int st = prep_state(s);
    if (st) return st;
    if ((st = run_gradients(s, c, fp.limiter != 0, false))) return st;
    if ((st = launch_stage(s, c, fp, 0, s->R))) return st;
    const Retire off{0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, nullptr, nullptr};
    HIPCHK(s, launch_resnorm(s->stream, s->R, s->n, s->nchunk, s->chunk_beg, s->part, s->ncase,
                             s->chunk_ptr, s->inv_nupd + (fp.kobc ? s->ncase : 0), s->wctr, 2,
                             s->wres, off, s->case_of, s->tile_active, s->tile_prec));
    return QL_OK;
}

int ql_wall_distance(ql_solver *s, double *d) {
    int st = ensure_ready(s, false);
    if (st) return st;
    if (!d) return fail(s, QL_EINVAL, "output is NULL");
    (void)hipSetDevice(s->device);
    HIPCHK(s, launch_wall_distance(s->stream, s->n, s->xy, s->case_of, s->dwall_lo, s->wall,
                                   s->tmp));
    std::vector<double> h(s->n);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->tmp, sizeof(double) * s->n, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int p = 0; p < s->n; ++p) d[s->perm[p]] = h[p];
    return QL_OK;
}

int ql_warm_start(ql_solver *s, ql_mlp *m, const float *X, const float *out_scale,
                  double rel_floor, double *res_cold, double *res_warm, int32_t *used) {
    int st = ensure_ready(s, false);
    if (st) return st;
    if (!ql::mlp_ready(m)) return fail(s, QL_EINVAL, "the network is not usable (no weights?)");
    if (!X || !out_scale) return fail(s, QL_EINVAL, "null features or output scale");
    if (ql::mlp_width(m, 1) != 4)
        return fail(s, QL_EINVAL, "the network must output 4 values (rho, u1, u2, p)");
    if (!(rel_floor > 0.0 && rel_floor < 1.0)) return fail(s, QL_EINVAL, "floor must lie in (0, 1)");
    (void)hipSetDevice(s->device);
    const int n = s->n, nc = s->ncase;
    // network output (caller order, FP32 [n][4]) into the residual buffer
    float *Y = reinterpret_cast<float *>(s->R);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if ((st = ql_mlp_forward(m, X, Y, n)))
        return fail(s, st, "network inference failed: %s", ql_mlp_last_error(m));
    HIPCHK(s, hipStreamSynchronize(ql::mlp_stream(m)));
    WarmScale sc;
    for (int k = 0; k < 4; ++k) {
        sc.mean[k] = out_scale[k];
        sc.std[k] = out_scale[4 + k];
    }
    sc.floor = rel_floor;
    if ((st = upload_freestream(s))) return st;
    HIPCHK(s, launch_warm_state(s->stream, n, s->dperm, s->kind, s->nrm, s->case_of, s->uinf, Y,
                                sc, s->prm.gamma, s->tmp));
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    HIPCHK(s, hipMemcpyAsync(s->wctr, &s->zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    // warm candidate: its stage-1 residual norms (row 0); a positivity or
    // finiteness failure rejects every case in which a point failed
    HIPCHK(s, hipMemcpyAsync(s->U, s->tmp, sizeof(double) * 4 * n, hipMemcpyDeviceToDevice,
                             s->stream));
    if ((st = reset_case_err(s))) return st;
    if ((st = warm_eval(s, c, fp))) return st;
    std::vector<ErrWord> cew(nc);
    HIPCHK(s, hipMemcpyAsync(cew.data(), s->case_err, sizeof(ErrWord) * nc, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if ((st = reset_case_err(s))) return st;
    // cold start: freestream (row 1); failures here are errors
    HIPCHK(s, launch_freestream(s->stream, n, s->nrm, s->kind, s->case_of, s->uinf, s->U));
    if ((st = warm_eval(s, c, fp))) return st;
    std::vector<double> rows((size_t)8 * nc);
    HIPCHK(s, hipMemcpyAsync(rows.data(), s->wres, sizeof(double) * rows.size(),
                             hipMemcpyDeviceToHost, s->stream));
    if ((st = sync_and_check(s, "warm_start (freestream)"))) return st;
    std::vector<uint8_t> sel(nc, 0);
    for (int k = 0; k < nc; ++k) {
        const double w = rows[4 * k], cold = rows[(size_t)4 * nc + 4 * k];
        sel[k] = (err_code(cew[k]) == kErrNone && std::isfinite(w) && w <= cold) ? 1 : 0;
        if (res_warm) std::copy(&rows[4 * k], &rows[4 * k] + 4, res_warm + 4 * k);
        if (res_cold) std::copy(&rows[(size_t)4 * nc + 4 * k], &rows[(size_t)4 * nc + 4 * k] + 4,
                                res_cold + 4 * k);
        if (used) used[k] = sel[k];
    }
    HIPCHK(s, hipMemcpyAsync(s->wsel, sel.data(), nc, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, launch_select_state(s->stream, n, s->case_of, s->wsel, s->tmp, s->U));
    if ((st = prep_state(s))) return st;
    st = sync_and_check(s, "warm_start");
    s->has_state = (st == QL_OK);
    s->has_eval = s->has_res = false;
    return st;
}

// --- autotuning of the LDS budgets ------------------------------------------

static std::string tune_key(const ql_solver *s) {
    char buf[128];
    const int lg = (int)std::lround(std::log2((double)std::max(s->n, 1)));
    const int kbar = (int)std::lround((double)s->nnz / std::max(s->n, 1));
    std::snprintf(buf, sizeof buf, "%s/lim%d/n2^%d/k%d", s->prm.precision ? "mixed" : "fp64",
                  s->prm.limiter, lg, kbar);
    return buf;
}

// entry lines of a cache file: "key": {"flux_lds": F, "grad_lds": G, ...}
static bool cache_lookup(const char *path, const std::string &key, int *f, int *g) {
    FILE *fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    const std::string head = "\"" + key + "\":";
    while (!found && std::fgets(line, sizeof line, fp)) {
        const char *p = std::strstr(line, head.c_str());
        if (!p) continue;
        const char *a = std::strstr(p, "\"flux_lds\":"), *b = std::strstr(p, "\"grad_lds\":");
        if (a && b && std::sscanf(a + 11, "%d", f) == 1 && std::sscanf(b + 11, "%d", g) == 1)
            found = true;
    }
    std::fclose(fp);
    return found;
}

static bool cache_store(const char *path, const std::string &key, const std::string &entry) {
    std::vector<std::string> keep;
    if (FILE *fp = std::fopen(path, "r")) {
        char line[512];
        const std::string head = "\"" + key + "\":";
        while (std::fgets(line, sizeof line, fp)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
            if (l.empty() || l == "{" || l == "}" || l.find(head) != std::string::npos) continue;
            keep.push_back(l);
        }
        std::fclose(fp);
    }
    keep.push_back(entry);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return false;
    std::fprintf(fp, "{\n");
    for (size_t i = 0; i < keep.size(); ++i)
        std::fprintf(fp, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    std::fprintf(fp, "}\n");
    const bool ok = std::fclose(fp) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

int ql_autotune(ql_solver *s, const char *cache_path, int32_t *chosen) {
    int st = ensure_ready(s, true);
    if (st) return st;
    (void)hipSetDevice(s->device);
    const std::string key = tune_key(s);
    int bf = 0, bg = 0;
    if (cache_path && cache_lookup(cache_path, key, &bf, &bg)) {
        ql_params p = s->prm;
        p.flux_lds = bf;
        p.grad_lds = bg;
        if ((st = ql_set_params(s, &p))) return st;
        if (chosen) {
            chosen[0] = bf;
            chosen[1] = bg;
        }
        return QL_OK;
    }
    const DevCloud c = dev_cloud(s);
    const FlowParams fp = flow_params(s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(s, hipEventCreate(&e0));
    HIPCHK(s, hipEventCreate(&e1));
    const bool was_timing = s->timing;
    s->timing = false;
    auto timed = [&](auto &&enqueue, int reps, double *us) -> int {
        int r = enqueue();  // warm-up
        if (r) return r;
        HIPCHK(s, hipEventRecord(e0, s->stream));
        for (int k = 0; k < reps; ++k)
            if ((r = enqueue())) return r;
        HIPCHK(s, hipEventRecord(e1, s->stream));
        HIPCHK(s, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
        *us = 1e3 * ms / reps;
        return QL_OK;
    };
    const int flux_c[] = {16, 24 << 10, 32 << 10, 40 << 10, 48 << 10, 52 << 10, 64 << 10, 80 << 10};
    const int grad_c[] = {16, 12 << 10, 16 << 10, 20 << 10, 22 << 10, 24 << 10, 28 << 10,
                          32 << 10};
    const ql_params saved = s->prm;
    double best_f = 1e30, best_g = 1e30, us = 0.0;
    if ((st = reset_err(s)) || (st = prep_state(s)) || (st = run_gradients(s, c, fp.limiter != 0, false)))
        goto done;
    for (int b : flux_c) {
        s->prm.flux_lds = b;
        if ((st = timed([&] { return launch_stage(s, c, fp, 0, s->R); }, 5, &us))) goto done;
        if (us < best_f) {
            best_f = us;
            bf = b;
        }
    }
    s->prm.flux_lds = saved.flux_lds;
    for (int b : grad_c) {
        s->prm.grad_lds = b;
        if ((st = timed([&] { return run_gradients(s, c, fp.limiter != 0, false); }, 3, &us))) goto done;
        if (us < best_g) {
            best_g = us;
            bg = b;
        }
    }
done:
    s->prm = saved;
    s->timing = was_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if ((st = sync_and_check(s, "autotune"))) return st;
    s->has_eval = false;
    s->prm.flux_lds = bf;
    s->prm.grad_lds = bg;
    s->graph_qcur = -1;  // a captured iteration holds the old budgets
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
    if (chosen) {
        chosen[0] = bf;
        chosen[1] = bg;
    }
    if (cache_path) {
        char entry[256];
        std::snprintf(entry, sizeof entry,
                      "\"%s\": {\"flux_lds\": %d, \"grad_lds\": %d, \"flux_us\": %.1f, "
                      "\"grad_us\": %.1f}",
                      key.c_str(), bf, bg, best_f, best_g);
        if (!cache_store(cache_path, key, entry))
            return fail(s, QL_EINVAL, "cannot write the tuning cache %s", cache_path);
    }
    return QL_OK;
}

int ql_batch_forces(ql_solver *s, double *cl, double *cd) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!cl || !cd) return fail(s, QL_EINVAL, "null output");
    (void)hipSetDevice(s->device);
    for (int c = 0; c < s->ncase; ++c)
        if ((st = case_forces(s, c, &cl[c], &cd[c]))) return st;
    return QL_OK;
}

int ql_batch_info(const ql_solver *s, int32_t *ncase) {
    if (!s || !s->has_cloud) return QL_ESTATE;
    if (ncase) *ncase = s->ncase;
    return QL_OK;
}

int ql_batch_status(const ql_solver *s, int32_t *status) {
    if (!s || !status) return QL_EINVAL;
    if (!s->has_cloud) return QL_ESTATE;
    for (int c = 0; c < s->ncase; ++c)
        status[c] = (c < (int)s->case_status.size()) ? s->case_status[c] : QL_OK;
    return QL_OK;
}

int ql_set_progress(ql_solver *s, ql_progress_fn fn, void *user) {
    if (!s) return QL_EINVAL;
    s->progress = fn;
    s->progress_user = user;
    return QL_OK;
}

int ql_batch_run(ql_solver *s, double drop, int32_t max_iter, int32_t check_every, int32_t graph,
                 const double *ref_res, int32_t *iters_out, double *res_out) {
    int st = ensure_ready(s, true);
    if (st) return st;
    if (!(drop > 0.0) || max_iter < 0 || check_every < 1)
        return fail(s, QL_EINVAL, "need drop > 0, max_iter >= 0, check_every >= 1");
    if (ref_res)
        for (int c = 0; c < s->ncase; ++c)
            if (!(ref_res[c] > 0.0) || !std::isfinite(ref_res[c]))
                return fail(s, QL_EINVAL, "reference residual of case %d must be > 0", c);
    (void)hipSetDevice(s->device);
    const int nc = s->ncase, ntile = num_flux_tiles(s->n);
    const int block = std::min(check_every, std::max(max_iter, 1));
    if ((st = ensure_history(s, block))) return st;
    // device retirement state: every case active, no reference yet (or the
    // caller's), no iterations, no failure
    std::vector<uint8_t> active(nc, 1), tile(ntile, 1);
    std::vector<double> ref(nc, -1.0), last((size_t)4 * nc, 0.0);
    if (ref_res) ref.assign(ref_res, ref_res + nc);
    std::vector<int> iters(nc, 0);
    std::vector<ErrWord> cerr(nc, kErrClear);
    std::vector<int32_t> status(nc, QL_OK);
    const double drop_h = drop;
    HIPCHK(s, hipMemcpyAsync(s->case_active, active.data(), nc, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->tile_active, tile.data(), ntile, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->bt_ref, ref.data(), sizeof(double) * nc, hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipMemcpyAsync(s->bt_last, last.data(), sizeof(double) * 4 * nc,
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->bt_iters, iters.data(), sizeof(int) * nc, hipMemcpyHostToDevice,
                             s->stream));
    HIPCHK(s, hipMemcpyAsync(s->bt_drop, &drop_h, sizeof(double), hipMemcpyHostToDevice,
                             s->stream));
    // mixed precision with a switch: every case starts with FP32 fluxes
    const bool hybrid = s->prm.precision == 1 && s->prm.mixed_switch > 0.0 && s->prm.order == 2;
    std::vector<int> swit(nc, -1);
    const double sw_h = s->prm.mixed_switch;
    if (hybrid) {
        const std::vector<uint8_t> ones_c(nc, 1), ones_t(ntile, 1);
        HIPCHK(s, hipMemcpyAsync(s->case_prec, ones_c.data(), nc, hipMemcpyHostToDevice,
                                 s->stream));
        HIPCHK(s, hipMemcpyAsync(s->tile_prec, ones_t.data(), ntile, hipMemcpyHostToDevice,
                                 s->stream));
        HIPCHK(s, hipMemcpyAsync(s->bt_swit, swit.data(), sizeof(int) * nc, hipMemcpyHostToDevice,
                                 s->stream));
        HIPCHK(s, hipMemcpyAsync(s->bt_switch, &sw_h, sizeof(double), hipMemcpyHostToDevice,
                                 s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));  // the host vectors go out of scope
    }
    s->hybrid = hybrid;
    if ((st = reset_err(s)) || (st = reset_case_err(s))) return st;
    const FlowParams fp = flow_params(s);
    // the iterations enqueued below retire cases on the device at the
    // iteration they converge, diverge or fail; the host only looks between
    // windows of check_every iterations, to stop once no case is active
    s->retire_on = true;
    s->live_on = false;
    int done = 0, nactive = nc, listed = nc;
    while (done < max_iter && nactive > 0) {
        const int k = std::min(block, max_iter - done);
        if ((st = reset_counter(s))) break;
        if (graph) {
            if ((st = capture_iteration(s))) break;
            for (int it = 0; it < k && !st; ++it)
                if (hipGraphLaunch(s->graph, s->stream) != hipSuccess)
                    st = fail(s, QL_EDEVICE, "graph launch failed");
            if (st) break;
        } else {
            const DevCloud cw = dev_cloud(s);
            for (int it = 0; it < k && !st; ++it) st = enqueue_iteration(s, cw, fp, block, s->reshist);
            if (st) break;
        }
        HIPCHK(s, hipMemcpyAsync(active.data(), s->case_active, nc, hipMemcpyDeviceToHost,
                                 s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        harvest_timing(s);
        nactive = (int)std::count(active.begin(), active.end(), (uint8_t)1);
        done += k;
        if (s->progress) s->progress(s->progress_user, done, nactive);
        if (nactive > 0 && nactive < listed && done < max_iter) {
            // cases retired in this window: from now on the tiled sweeps
            // launch over the tiles that still hold an active case (tiles
            // only ever leave the set during a run, and a listed tile that
            // retires later is skipped by its tile_active flag as before)
            tile.resize(ntile);
            HIPCHK(s, hipMemcpyAsync(tile.data(), s->tile_active, ntile, hipMemcpyDeviceToHost,
                                     s->stream));
            HIPCHK(s, hipStreamSynchronize(s->stream));
            s->tile_list_h.clear();
            for (int t = 0; t < ntile; ++t)
                if (tile[t]) s->tile_list_h.push_back(t);
            if (s->tile_list_h.empty()) s->tile_list_h.push_back(0);
            s->ntile_live = (int)s->tile_list_h.size();
            HIPCHK(s, hipMemcpyAsync(s->tile_list, s->tile_list_h.data(),
                                     sizeof(int) * s->tile_list_h.size(), hipMemcpyHostToDevice,
                                     s->stream));
            s->live_on = true;
            listed = nactive;
        }
    }
    s->retire_on = false;
    s->live_on = false;
    s->hybrid = false;
    if (st) return st;
    if (hybrid)
        HIPCHK(s, hipMemcpyAsync(swit.data(), s->bt_swit, sizeof(int) * nc, hipMemcpyDeviceToHost,
                                 s->stream));
    HIPCHK(s, hipMemcpyAsync(iters.data(), s->bt_iters, sizeof(int) * nc, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipMemcpyAsync(last.data(), s->bt_last, sizeof(double) * 4 * nc,
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(ref.data(), s->bt_ref, sizeof(double) * nc, hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipMemcpyAsync(cerr.data(), s->case_err, sizeof(ErrWord) * nc,
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int cs = 0; cs < nc; ++cs) {
        const int code = err_code(cerr[cs]);
        if (code == kErrPositivity) status[cs] = QL_EPOSITIVITY;
        else if (code == kErrNonFinite) status[cs] = QL_ENONFINITE;
        else if (code != kErrNone) return err_status(s, cerr[cs], "batch_run");
        else if (iters[cs] > 0 && !(last[4 * cs] <= kDiverged * ref[cs]))
            status[cs] = QL_EDIVERGED;
    }
    // leave every case active for later calls, and rebuild the start-of-
    // iteration data (q, time step, Un) from U: retired cases' q buffers were
    // not kept current.  Only a case that failed may fail here.
    std::fill(active.begin(), active.end(), 1);
    std::fill(tile.begin(), tile.end(), 1);
    HIPCHK(s, hipMemcpyAsync(s->case_active, active.data(), nc, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->tile_active, tile.data(), ntile, hipMemcpyHostToDevice, s->stream));
    if ((st = reset_case_err(s)) || (st = prep_state(s))) return st;
    HIPCHK(s, hipMemcpyAsync(cerr.data(), s->case_err, sizeof(ErrWord) * nc,
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int cs = 0; cs < nc; ++cs)
        if (err_code(cerr[cs]) != kErrNone && status[cs] == QL_OK)
            return err_status(s, cerr[cs], "batch_run");
    if ((st = reset_err(s)) || (st = reset_case_err(s))) return st;
    s->has_eval = false;
    s->case_status = status;
    s->case_switch.assign(swit.begin(), swit.end());
    s->last_res = last;
    s->has_res = done > 0;
    if (iters_out) std::copy(iters.begin(), iters.end(), iters_out);
    if (res_out) std::copy(last.begin(), last.end(), res_out);
    return QL_OK;
}

int ql_batch_switched(const ql_solver *s, int32_t *iter) {
    if (!s || !iter) return QL_EINVAL;
    if (!s->has_cloud) return QL_ESTATE;
    for (int c = 0; c < s->ncase; ++c)
        iter[c] = (c < (int)s->case_switch.size()) ? s->case_switch[c] : -1;
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
    if (int st = settle(const_cast<ql_solver *>(s))) return st;
    if (total_ms) *total_ms = s->tsum[which];
    if (count) *count = s->tcnt[which];
    return QL_OK;
}

}  // extern "C"
