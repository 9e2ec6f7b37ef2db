// Host runtime of the warm-start network (the ql_mlp_* entry points of
// include/qlskum.h): owns the FP32 master weights, the Adam moments, the
// bf16 operand copies and the activation workspace of one network, and
// sequences the kernels of qlskum_mlp.hip for inference and training.
#include "../../include/qlskum.h"
#include "qlskum_mlp_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

using namespace ql;

struct ql_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    std::string err;

    std::vector<int> widths;  // w_0 .. w_L
    int64_t max_batch = 0;
    int np = 0;
    std::vector<int> woff;  // offset of W_l in the flat vector (b_l follows)
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    std::vector<bf16 *> Wb, WbT;  // per layer: W_l and W_l^T in bf16
    std::vector<bf16 *> act;      // a_0 .. a_{L-1} in bf16, [max_batch][w_l]
    float *y = nullptr;           // [max_batch][w_L]
    bf16 *d[2] = {nullptr, nullptr};
    float *part = nullptr, *loss = nullptr;
    float *gpart = nullptr;  // split-K partial products of the weight gradients
    int64_t t = 0;  // Adam steps taken
    bool has_weights = false;
};

namespace {

int mfail(ql_mlp *m, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    m->err = buf;
    if (code == QL_EDEVICE) m->poisoned = true;
    return code;
}

#define MCHK(m, call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return mfail((m), QL_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t malloc_n(T **p, size_t count) {
    *p = nullptr;
    return hipMalloc((void **)p, (count ? count : 1) * sizeof(T));
}

template <typename T>
void free_p(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

int nlayers(const ql_mlp *m) { return (int)m->widths.size() - 1; }

int ready(ql_mlp *m, bool need_weights) {
    if (!m) return QL_EINVAL;
    if (m->poisoned) return QL_EDEVICE;
    if (need_weights && !m->has_weights) return mfail(m, QL_ESTATE, "set the weights first");
    (void)hipSetDevice(m->device);
    return QL_OK;
}

// bf16 operand copies of every layer's weights
int refresh_bf16(ql_mlp *m) {
    for (int l = 0; l < nlayers(m); ++l)
        MCHK(m, launch_weights_bf16(m->stream, m->widths[l], m->widths[l + 1], m->w + m->woff[l],
                                    m->Wb[l], m->WbT[l]));
    return QL_OK;
}

// forward pass of rows [0, n) of X (device FP32 [n][w_0]) into m->act, m->y
int forward(ql_mlp *m, const float *X, int64_t n) {
    const int L = nlayers(m);
    MCHK(m, launch_to_bf16(m->stream, n, m->widths[0], m->widths[0], X, m->act[0]));
    for (int l = 0; l < L; ++l) {
        const int fi = m->widths[l], fo = m->widths[l + 1];
        const float *bias = m->w + m->woff[l] + (size_t)fi * fo;
        if (l + 1 < L)
            MCHK(m, launch_mfma_gemm(m->stream, kEpiBiasTanh, true, true, (int)n, fo, fi,
                                     m->act[l], fi, m->WbT[l], fi, bias, nullptr, nullptr,
                                     m->act[l + 1], fo));
        else
            MCHK(m, launch_mfma_gemm(m->stream, kEpiBias, true, true, (int)n, fo, fi, m->act[l],
                                     fi, m->WbT[l], fi, bias, nullptr, m->y, nullptr, fo));
    }
    return QL_OK;
}

// forward + backward of one batch; gradient (flat) into m->g, sum of squared
// errors into m->loss[0]
int gradient(ql_mlp *m, const float *X, const float *T, int64_t n) {
    int st = forward(m, X, n);
    if (st) return st;
    const int L = nlayers(m);
    const int wL = m->widths[L];
    const int64_t cnt = n * wL;
    MCHK(m, launch_loss(m->stream, cnt, (float)(2.0 / (double)cnt), m->y, T, m->d[0], m->part,
                        m->loss));
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int fi = m->widths[l], fo = m->widths[l + 1];
        float *gW = m->g + m->woff[l];
        // dW_l = a_{l-1}^T d_l: op(A)(i, r) = act[r*fi + i], op(B)(r, j) = d[r*fo + j];
        // the inner dimension is the batch, so the product is split along it
        MCHK(m, launch_mfma_gemm_splitk(m->stream, false, false, fi, fo, (int)n, m->act[l], fi,
                                        m->d[cur], fo, m->gpart, gW, fo));
        MCHK(m, launch_colsum(m->stream, n, fo, m->d[cur], gW + (size_t)fi * fo));
        if (l > 0) {
            // d_{l-1} = (d_l W_l^T) * (1 - a_{l-1}^2): op(B)(j, i) = Wb[i*fo + j]
            MCHK(m, launch_mfma_gemm(m->stream, kEpiTanhGrad, true, true, (int)n, fi, fo,
                                     m->d[cur], fo, m->Wb[l], fo, nullptr, m->act[l], nullptr,
                                     m->d[1 - cur], fi));
            cur = 1 - cur;
        }
    }
    return QL_OK;
}

int check_batch(ql_mlp *m, const void *X, const void *T, int64_t n, bool need_t) {
    if (!X || (need_t && !T)) return mfail(m, QL_EINVAL, "null device pointer");
    if (n < 1 || n > m->max_batch)
        return mfail(m, QL_EINVAL, "batch of %lld rows outside [1, %lld]", (long long)n,
                     (long long)m->max_batch);
    return QL_OK;
}

}  // namespace

extern "C" {

int ql_mlp_create(ql_mlp **out, int32_t device, void *hip_stream, const int32_t *widths,
                  int32_t nwidth, int64_t max_batch) {
    if (!out) return QL_EINVAL;
    *out = nullptr;
    if (!widths || nwidth < 2 || max_batch < 1 || max_batch > (int64_t)1 << 26) return QL_EINVAL;
    for (int i = 0; i < nwidth; ++i)
        if (widths[i] < 1 || widths[i] > 4096) return QL_EINVAL;
    ql_mlp *m = new (std::nothrow) ql_mlp();
    if (!m) return QL_ENOMEM;
    m->device = device;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
        hipSetDevice(device) != hipSuccess) {
        delete m;
        return QL_EDEVICE;
    }
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&m->stream) != hipSuccess) {
            delete m;
            return QL_EDEVICE;
        }
        m->own_stream = true;
    }
    m->widths.assign(widths, widths + nwidth);
    m->max_batch = max_batch;
    int maxw = 0;
    for (int l = 0; l + 1 < nwidth; ++l) {
        m->woff.push_back(m->np);
        m->np += widths[l] * widths[l + 1] + widths[l + 1];
    }
    for (int i = 0; i < nwidth; ++i) maxw = std::max(maxw, (int)widths[i]);
    bool okm = malloc_n(&m->w, m->np) == hipSuccess && malloc_n(&m->m, m->np) == hipSuccess &&
               malloc_n(&m->v, m->np) == hipSuccess && malloc_n(&m->g, m->np) == hipSuccess;
    m->Wb.assign(nwidth - 1, nullptr);
    m->WbT.assign(nwidth - 1, nullptr);
    m->act.assign(nwidth - 1, nullptr);
    for (int l = 0; okm && l + 1 < nwidth; ++l) {
        okm = malloc_n(&m->Wb[l], (size_t)widths[l] * widths[l + 1]) == hipSuccess &&
              malloc_n(&m->WbT[l], (size_t)widths[l] * widths[l + 1]) == hipSuccess &&
              malloc_n(&m->act[l], (size_t)max_batch * widths[l]) == hipSuccess;
    }
    const int64_t cnt = max_batch * widths[nwidth - 1];
    okm = okm && malloc_n(&m->y, (size_t)cnt) == hipSuccess &&
          malloc_n(&m->d[0], (size_t)max_batch * maxw) == hipSuccess &&
          malloc_n(&m->d[1], (size_t)max_batch * maxw) == hipSuccess &&
          malloc_n(&m->part, (size_t)((cnt + 255) / 256)) == hipSuccess &&
          malloc_n(&m->loss, 1) == hipSuccess;
    size_t gp = 0;
    for (int l = 0; l + 1 < nwidth; ++l) {
        const int nsl = gemm_splitk_slices(widths[l], widths[l + 1], (int)max_batch);
        if (nsl > 1) gp = std::max(gp, (size_t)nsl * widths[l] * widths[l + 1]);
    }
    okm = okm && (gp == 0 || malloc_n(&m->gpart, gp) == hipSuccess);
    if (!okm) {
        ql_mlp_destroy(m);
        return QL_ENOMEM;
    }
    *out = m;
    return QL_OK;
}

int ql_mlp_destroy(ql_mlp *m) {
    if (!m) return QL_OK;
    (void)hipSetDevice(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    free_p(m->w); free_p(m->m); free_p(m->v); free_p(m->g);
    for (auto &p : m->Wb) free_p(p);
    for (auto &p : m->WbT) free_p(p);
    for (auto &p : m->act) free_p(p);
    free_p(m->y); free_p(m->d[0]); free_p(m->d[1]); free_p(m->part); free_p(m->loss);
    free_p(m->gpart);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return QL_OK;
}

const char *ql_mlp_last_error(const ql_mlp *m) { return m ? m->err.c_str() : "null network"; }

int ql_mlp_num_params(const ql_mlp *m, int64_t *np) {
    if (!m || !np) return QL_EINVAL;
    *np = m->np;
    return QL_OK;
}

int ql_mlp_set_weights(ql_mlp *m, const float *w) {
    int st = ready(m, false);
    if (st) return st;
    if (!w) return mfail(m, QL_EINVAL, "weights are NULL");
    for (int i = 0; i < m->np; ++i)
        if (!std::isfinite(w[i])) return mfail(m, QL_ENONFINITE, "weight %d is not finite", i);
    MCHK(m, hipMemcpyAsync(m->w, w, sizeof(float) * m->np, hipMemcpyHostToDevice, m->stream));
    MCHK(m, hipMemsetAsync(m->m, 0, sizeof(float) * m->np, m->stream));
    MCHK(m, hipMemsetAsync(m->v, 0, sizeof(float) * m->np, m->stream));
    m->t = 0;
    st = refresh_bf16(m);
    if (st) return st;
    MCHK(m, hipStreamSynchronize(m->stream));  // the host array may go away
    m->has_weights = true;
    return QL_OK;
}

int ql_mlp_get_weights(ql_mlp *m, float *w) {
    int st = ready(m, true);
    if (st) return st;
    if (!w) return mfail(m, QL_EINVAL, "output is NULL");
    MCHK(m, hipMemcpyAsync(w, m->w, sizeof(float) * m->np, hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    return QL_OK;
}

int ql_mlp_forward(ql_mlp *m, const float *X, float *Y, int64_t n) {
    int st = ready(m, true);
    if (st) return st;
    if (n < 0 || (n > 0 && (!X || !Y))) return mfail(m, QL_EINVAL, "bad forward arguments");
    const int w0 = m->widths.front(), wL = m->widths.back();
    for (int64_t r = 0; r < n; r += m->max_batch) {
        const int64_t b = std::min(m->max_batch, n - r);
        if ((st = forward(m, X + r * w0, b))) return st;
        MCHK(m, hipMemcpyAsync(Y + r * wL, m->y, sizeof(float) * b * wL,
                               hipMemcpyDeviceToDevice, m->stream));
    }
    return QL_OK;
}

int ql_mlp_gradient(ql_mlp *m, const float *X, const float *T, int64_t n, float *grad,
                    double *loss) {
    int st = ready(m, true);
    if (st) return st;
    if ((st = check_batch(m, X, T, n, true))) return st;
    if ((st = gradient(m, X, T, n))) return st;
    float l = 0.0f;
    if (grad)
        MCHK(m, hipMemcpyAsync(grad, m->g, sizeof(float) * m->np, hipMemcpyDeviceToHost,
                               m->stream));
    MCHK(m, hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    if (loss) *loss = (double)l / (double)(n * m->widths.back());
    return QL_OK;
}

int ql_mlp_train_step(ql_mlp *m, const float *X, const float *T, int64_t n, float lr,
                      double *loss) {
    int st = ready(m, true);
    if (st) return st;
    if ((st = check_batch(m, X, T, n, true))) return st;
    if (!(lr > 0.0f) || !std::isfinite(lr)) return mfail(m, QL_EINVAL, "bad learning rate");
    if ((st = gradient(m, X, T, n))) return st;
    m->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)m->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)m->t)));
    MCHK(m, launch_adam(m->stream, m->np, lr, (float)b1, (float)b2, 1e-8f, c1, c2, m->g, m->w,
                        m->m, m->v));
    if ((st = refresh_bf16(m))) return st;
    if (loss) {
        float l = 0.0f;
        MCHK(m, hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
        *loss = (double)l / (double)(n * m->widths.back());
    }
    return QL_OK;
}

int ql_mlp_sync(ql_mlp *m) {
    int st = ready(m, false);
    if (st) return st;
    MCHK(m, hipStreamSynchronize(m->stream));
    return QL_OK;
}

}  // extern "C"

// for the solver's warm start
namespace ql {
hipStream_t mlp_stream(const ql_mlp *m) { return m->stream; }
int mlp_width(const ql_mlp *m, int end) { return end ? m->widths.back() : m->widths.front(); }
bool mlp_ready(const ql_mlp *m) { return m && !m->poisoned && m->has_weights; }
}  // namespace ql
