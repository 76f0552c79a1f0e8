// Small dense products inside one workgroup (operands in LDS or global
// memory, FP64 MFMA), for the one-workgroup solver kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace ttr {
namespace {

typedef double ldsmm_d4 __attribute__((ext_vector_type(4)));

// C(M x N) = alpha op(A)(M x K) op(B)(K x N) + beta Cin, row-major with
// leading dimensions lda/ldb/ldc/ldci; op(A) = A or A^T (TA), op(B) = B or
// B^T (TB).  16 x 16 blocks are dealt round-robin to the wavefronts of the
// workgroup; f64 MFMA layout: A lane (r, q) = op(A)[m0+r][k+q], B lane =
// op(B)[k+q][n0+r], D register j = row q + 4j, column r.
template <bool TA, bool TB>
__device__ void lds_gemm(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                         int M, int N, int K, double alpha = 1.0, const double *Cin = nullptr,
                         int ldci = 0, double beta = 0.0) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int bm = (M + 15) / 16, bn = (N + 15) / 16;
  for (int blk = wave; blk < bm * bn; blk += nw) {
    const int m0 = (blk / bn) * 16, n0 = (blk % bn) * 16;
    ldsmm_d4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + q;
      const int m = m0 + r, n = n0 + r;
      double a = 0.0, b = 0.0;
      if (k < K && m < M) a = TA ? A[k * lda + m] : A[m * lda + k];
      if (k < K && n < N) b = TB ? B[n * ldb + k] : B[k * ldb + n];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = m0 + q + 4 * j, col = n0 + r;
      if (row < M && col < N) {
        double v = alpha * acc[j];
        if (beta != 0.0) v += beta * Cin[row * ldci + col];
        C[row * ldc + col] = v;
      }
    }
  }
}

}  // namespace
}  // namespace ttr
