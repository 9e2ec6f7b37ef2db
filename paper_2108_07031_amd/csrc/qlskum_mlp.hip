// Warm-start network kernels for gfx950: a multilayer perceptron
//   a_0 = x,  z_l = a_{l-1} W_l + b_l,  a_l = tanh(z_l) (hidden),  y = z_L
// evaluated and trained with bfloat16 operands on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation); bias, tanh, loss, the
// gradient sums and Adam in FP32.
//
// Product kernel: one wavefront computes one 16 x 16 block of
// C = op(A) op(B) (M x N, inner dimension K) in steps of 32 along K.  With
// the gfx950 16x16x32 layout, lane l holds
//   A[row l%16][k 8(l/16) .. 8(l/16)+7],  B[k 8(l/16) .. +7][col l%16],
//   C[rows 4(l/16) .. 4(l/16)+3][col l%16].
// Operands are addressed through (pointer, leading dimension, transposed):
// element (r, k) of op(P) is P[r*ld + k] (k contiguous) or P[k*ld + r].
#include "qlskum_mlp_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace ql {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;  // wavefronts (output blocks) per workgroup

// 8 consecutive-k elements of row r of op(P), zero outside r < R, k < K
template <bool KCONTIG>
__device__ __forceinline__ bf16x8 load_frag(const bf16 *__restrict__ P, int ld, int r, int k0,
                                            int R, int K) {
    bf16x8 v;
    if (KCONTIG && r < R && k0 + 8 <= K && (ld & 7) == 0) {
        v = *reinterpret_cast<const bf16x8 *>(P + (size_t)r * ld + k0);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + i;
            v[i] = (r < R && k < K) ? P[KCONTIG ? (size_t)r * ld + k : (size_t)k * ld + r]
                                    : (bf16)0.0f;
        }
    }
    return v;
}

}  // namespace

// C = op(A) op(B) with an epilogue:
//   kEpiStore     C32[m, n] = acc
//   kEpiBias      C32[m, n] = acc + bias[n]
//   kEpiBiasTanh  C16[m, n] = bf16(tanh(acc + bias[n]))
//   kEpiTanhGrad  C16[m, n] = bf16(acc * (1 - a^2)),  a = act[m, n] (bf16)
// A_KC: element (m, k) of op(A) is A[m*lda + k] (else A[k*lda + m]);
// B_NC: element (k, n) of op(B) is B[n*ldb + k] (else B[k*ldb + n]).
template <bool A_KC, bool B_NC, int EPI>
__global__ void __launch_bounds__(64 * kWaves)
    k_mfma_gemm(int M, int N, int K, const bf16 *__restrict__ A, int lda,
                const bf16 *__restrict__ B, int ldb, const float *__restrict__ bias,
                const bf16 *__restrict__ act, float *__restrict__ C32, bf16 *__restrict__ C16,
                int ldc) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int ntn = (N + 15) / 16;
    const int ntiles = ((M + 15) / 16) * ntn;
    if (tile >= ntiles) return;  // whole wavefront leaves together
    const int tm = tile / ntn, tn = tile % ntn;
    const int r = tm * 16 + (lane & 15);  // row of op(A) this lane loads
    const int c = tn * 16 + (lane & 15);  // column of op(B) this lane loads
    const int kq = 8 * (lane >> 4);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = load_frag<A_KC>(A, lda, r, k0 + kq, M, K);
        const bf16x8 b = load_frag<B_NC>(B, ldb, c, k0 + kq, N, K);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    const int n = tn * 16 + (lane & 15);
    if (n >= N) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = tm * 16 + 4 * (lane >> 4) + i;
        if (m >= M) continue;
        const size_t o = (size_t)m * ldc + n;
        const float v = acc[i];
        if (EPI == kEpiStore) {
            C32[o] = v;
        } else if (EPI == kEpiBias) {
            C32[o] = v + bias[n];
        } else if (EPI == kEpiBiasTanh) {
            C16[o] = (bf16)tanhf(v + bias[n]);
        } else {
            const float a = (float)act[o];
            C16[o] = (bf16)(v * (1.0f - a * a));
        }
    }
}

hipError_t launch_mfma_gemm(hipStream_t st, int epi, bool a_kc, bool b_nc, int M, int N, int K,
                            const bf16 *A, int lda, const bf16 *B, int ldb, const float *bias,
                            const bf16 *act, float *C32, bf16 *C16, int ldc) {
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    if (tiles == 0) return hipSuccess;
    const dim3 grid((tiles + kWaves - 1) / kWaves), block(64 * kWaves);
#define QL_GEMM(AK, BN, E)                                                                 \
    hipLaunchKernelGGL((k_mfma_gemm<AK, BN, E>), grid, block, 0, st, M, N, K, A, lda, B, ldb, \
                       bias, act, C32, C16, ldc)
#define QL_GEMM_EPI(AK, BN)                                    \
    switch (epi) {                                             \
    case kEpiStore: QL_GEMM(AK, BN, kEpiStore); break;         \
    case kEpiBias: QL_GEMM(AK, BN, kEpiBias); break;           \
    case kEpiBiasTanh: QL_GEMM(AK, BN, kEpiBiasTanh); break;   \
    default: QL_GEMM(AK, BN, kEpiTanhGrad); break;             \
    }
    if (a_kc && b_nc) { QL_GEMM_EPI(true, true) }
    else if (a_kc) { QL_GEMM_EPI(true, false) }
    else if (b_nc) { QL_GEMM_EPI(false, true) }
    else { QL_GEMM_EPI(false, false) }
#undef QL_GEMM_EPI
#undef QL_GEMM
    return hipGetLastError();
}

// Split-K form of the plain product (kEpiStore) for few output blocks and a
// long inner dimension -- the weight gradients a^T d, whose inner dimension
// is the batch: wavefront (slice, block) sums one 16 x 16 block over the
// kslice-long slice of K into part[slice][M][N], and k_gemm_reduce adds the
// slices in slice order (a fixed order: results do not depend on timing).
template <bool A_KC, bool B_NC>
__global__ void __launch_bounds__(64 * kWaves)
    k_mfma_gemm_splitk(int M, int N, int K, int kslice, const bf16 *__restrict__ A, int lda,
                       const bf16 *__restrict__ B, int ldb, float *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int ntn = (N + 15) / 16;
    const int ntiles = ((M + 15) / 16) * ntn;
    const int nsl = (K + kslice - 1) / kslice;
    if (item >= ntiles * nsl) return;  // whole wavefront leaves together
    const int sl = item / ntiles, tile = item % ntiles;
    const int tm = tile / ntn, tn = tile % ntn;
    const int r = tm * 16 + (lane & 15);
    const int c = tn * 16 + (lane & 15);
    const int kq = 8 * (lane >> 4);
    const int kb = sl * kslice, ke = min(K, kb + kslice);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        const bf16x8 a = load_frag<A_KC>(A, lda, r, k0 + kq, M, ke);
        const bf16x8 b = load_frag<B_NC>(B, ldb, c, k0 + kq, N, ke);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    const int n = tn * 16 + (lane & 15);
    if (n >= N) return;
    float *P = part + (size_t)sl * M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = tm * 16 + 4 * (lane >> 4) + i;
        if (m < M) P[(size_t)m * N + n] = acc[i];
    }
}

__global__ void __launch_bounds__(256) k_gemm_reduce(int M, int N, int nsl,
                                                     const float *__restrict__ part,
                                                     float *__restrict__ C, int ldc) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    float s = 0.0f;
    for (int sl = 0; sl < nsl; ++sl) s += part[(size_t)sl * M * N + idx];
    C[(size_t)(idx / N) * ldc + idx % N] = s;
}

int gemm_splitk_slices(int M, int N, int K) {
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    if (tiles == 0 || tiles > kSplitKMaxTiles || K < 2 * kSplitKSlice) return 1;
    return std::min(kSplitKMaxSlices, (K + kSplitKSlice - 1) / kSplitKSlice);
}

hipError_t launch_mfma_gemm_splitk(hipStream_t st, bool a_kc, bool b_nc, int M, int N, int K,
                                   const bf16 *A, int lda, const bf16 *B, int ldb, float *part,
                                   float *C32, int ldc) {
    const int nsl = gemm_splitk_slices(M, N, K);
    if (nsl <= 1)
        return launch_mfma_gemm(st, kEpiStore, a_kc, b_nc, M, N, K, A, lda, B, ldb, nullptr,
                                nullptr, C32, nullptr, ldc);
    // slices of a whole number of 32-deep steps, nsl of them covering K
    const int kslice = ((K + nsl - 1) / nsl + 31) / 32 * 32;
    const int nsl_used = (K + kslice - 1) / kslice;
    const int items = ((M + 15) / 16) * ((N + 15) / 16) * nsl_used;
    const dim3 grid((items + kWaves - 1) / kWaves), block(64 * kWaves);
    if (a_kc && b_nc)
        hipLaunchKernelGGL((k_mfma_gemm_splitk<true, true>), grid, block, 0, st, M, N, K, kslice,
                           A, lda, B, ldb, part);
    else if (a_kc)
        hipLaunchKernelGGL((k_mfma_gemm_splitk<true, false>), grid, block, 0, st, M, N, K, kslice,
                           A, lda, B, ldb, part);
    else if (b_nc)
        hipLaunchKernelGGL((k_mfma_gemm_splitk<false, true>), grid, block, 0, st, M, N, K, kslice,
                           A, lda, B, ldb, part);
    else
        hipLaunchKernelGGL((k_mfma_gemm_splitk<false, false>), grid, block, 0, st, M, N, K,
                           kslice, A, lda, B, ldb, part);
    hipLaunchKernelGGL(k_gemm_reduce, dim3((M * N + 255) / 256), dim3(256), 0, st, M, N, nsl_used,
                       part, C32, ldc);
    return hipGetLastError();
}

// FP32 -> bf16, row-major [n][w] with leading dimension ld (columns w..ld-1
// of the destination are set to zero).
__global__ void __launch_bounds__(256) k_to_bf16(int64_t n, int w, int ld,
                                                 const float *__restrict__ x,
                                                 bf16 *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * ld) return;
    const int64_t r = i / ld;
    const int c = (int)(i - r * ld);
    y[i] = (c < w) ? (bf16)x[r * w + c] : (bf16)0.0f;
}

hipError_t launch_to_bf16(hipStream_t st, int64_t n, int w, int ld, const float *x, bf16 *y) {
    const int64_t tot = n * ld;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, w, ld,
                       x, y);
    return hipGetLastError();
}

// Output error of the mean squared loss: dy = bf16(scale (y - t)) with
// scale = 2 / (n nout), and one partial sum of (y - t)^2 per workgroup
// (fixed-order tree).
__global__ void __launch_bounds__(256) k_loss(int64_t cnt, float scale,
                                              const float *__restrict__ y,
                                              const float *__restrict__ t,
                                              bf16 *__restrict__ dy, float *__restrict__ part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e2 = 0.0f;
    if (i < cnt) {
        const float d = y[i] - t[i];
        dy[i] = (bf16)(scale * d);
        e2 = d * d;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of part[0..np) in a fixed order (one workgroup)
__global__ void __launch_bounds__(256) k_sum(int np, const float *__restrict__ part,
                                             float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_loss(hipStream_t st, int64_t cnt, float scale, const float *y, const float *t,
                       bf16 *dy, float *part, float *out) {
    const unsigned nb = (unsigned)((cnt + 255) / 256);
    if (nb == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, cnt, scale, y, t, dy, part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, (int)nb, part, out);
    return hipGetLastError();
}

// Column sums of a bf16 matrix [n][w] into FP32 out[w]: one workgroup per
// column, fixed-order tree.
__global__ void __launch_bounds__(256) k_colsum(int64_t n, int w, const bf16 *__restrict__ d,
                                                float *__restrict__ out) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < n; r += 256) s += (float)d[r * w + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

hipError_t launch_colsum(hipStream_t st, int64_t n, int w, const bf16 *d, float *out) {
    hipLaunchKernelGGL(k_colsum, dim3(w), dim3(256), 0, st, n, w, d, out);
    return hipGetLastError();
}

// Adam (Kingma and Ba, 2015) on the FP32 master weights with bias-corrected
// moments: c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ void __launch_bounds__(256) k_adam(int np, float lr, float b1, float b2, float eps,
                                              float c1, float c2, const float *__restrict__ g,
                                              float *__restrict__ w, float *__restrict__ m,
                                              float *__restrict__ v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

hipError_t launch_adam(hipStream_t st, int np, float lr, float b1, float b2, float eps, float c1,
                       float c2, const float *g, float *w, float *m, float *v) {
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, st, np, lr, b1, b2, eps, c1,
                       c2, g, w, m, v);
    return hipGetLastError();
}

// bf16 operand copies of one layer's FP32 weights W [fi][fo] (row-major):
// Wb = W (row-major) and WbT = W^T (row-major [fo][fi]).
__global__ void __launch_bounds__(256) k_weights_bf16(int fi, int fo, const float *__restrict__ W,
                                                      bf16 *__restrict__ Wb,
                                                      bf16 *__restrict__ WbT) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= fi * fo) return;
    const int r = i / fo, c = i - r * fo;
    const bf16 v = (bf16)W[i];
    Wb[i] = v;
    WbT[(size_t)c * fi + r] = v;
}

hipError_t launch_weights_bf16(hipStream_t st, int fi, int fo, const float *W, bf16 *Wb,
                               bf16 *WbT) {
    hipLaunchKernelGGL(k_weights_bf16, dim3((fi * fo + 255) / 256), dim3(256), 0, st, fi, fo, W,
                       Wb, WbT);
    return hipGetLastError();
}

}  // namespace ql
