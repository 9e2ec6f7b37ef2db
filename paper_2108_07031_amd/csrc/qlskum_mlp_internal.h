// Internal interface between the warm-start network's host runtime and its
// HIP kernels.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ql {

typedef __bf16 bf16;

enum MlpEpilogue : int { kEpiStore = 0, kEpiBias = 1, kEpiBiasTanh = 2, kEpiTanhGrad = 3 };

// C (M x N, leading dimension ldc) = op(A) op(B) with inner dimension K on
// the bf16 matrix cores, FP32 accumulation, then the epilogue (see the
// kernel).  a_kc: element (m, k) of op(A) is A[m*lda + k], else A[k*lda + m];
// b_nc: element (k, n) of op(B) is B[n*ldb + k], else B[k*ldb + n].
hipError_t launch_mfma_gemm(hipStream_t st, int epi, bool a_kc, bool b_nc, int M, int N, int K,
                            const bf16 *A, int lda, const bf16 *B, int ldb, const float *bias,
                            const bf16 *act, float *C32, bf16 *C16, int ldc);
// The plain product (kEpiStore) split along K when it has at most
// kSplitKMaxTiles output blocks and K is long: up to kSplitKMaxSlices
// slices of at least kSplitKSlice, partial products in part (at least
// gemm_splitk_slices(M, N, K) * M * N floats), then added in slice order.
constexpr int kSplitKMaxTiles = 256, kSplitKMaxSlices = 64, kSplitKSlice = 256;
int gemm_splitk_slices(int M, int N, int K);
hipError_t launch_mfma_gemm_splitk(hipStream_t st, bool a_kc, bool b_nc, int M, int N, int K,
                                   const bf16 *A, int lda, const bf16 *B, int ldb, float *part,
                                   float *C32, int ldc);
hipError_t launch_to_bf16(hipStream_t st, int64_t n, int w, int ld, const float *x, bf16 *y);
// dy = bf16(scale (y - t)); *out = sum (y - t)^2 (part: >= ceil(cnt/256) floats)
hipError_t launch_loss(hipStream_t st, int64_t cnt, float scale, const float *y, const float *t,
                       bf16 *dy, float *part, float *out);
hipError_t launch_colsum(hipStream_t st, int64_t n, int w, const bf16 *d, float *out);
hipError_t launch_adam(hipStream_t st, int np, float lr, float b1, float b2, float eps, float c1,
                       float c2, const float *g, float *w, float *m, float *v);
hipError_t launch_weights_bf16(hipStream_t st, int fi, int fo, const float *W, bf16 *Wb,
                               bf16 *WbT);

}  // namespace ql
