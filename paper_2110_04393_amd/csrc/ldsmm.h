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
// op(B)[k+q][n0+r], D register j = row q + 4j, column r.  A dependent f64
// MFMA waits for its predecessor, so consecutive k-steps go to four
// accumulators (summed at the end) and each group of four steps loads its
// operands before its products.  Rows and columns past M and N read the last
// valid one (their results are not written); k-steps past K read zeros.
template <bool TA, bool TB>
__device__ void lds_gemm(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                         int M, int N, int K, double alpha = 1.0, const double *Cin = nullptr,
                         int ldci = 0, double beta = 0.0) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int bm = (M + 15) / 16, bn = (N + 15) / 16;
  for (int blk = wave; blk < bm * bn; blk += nw) {
    const int m0 = (blk / bn) * 16, n0 = (blk % bn) * 16;
    const int m = min(m0 + r, M - 1), n = min(n0 + r, N - 1);
    ldsmm_d4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = ldsmm_d4{0, 0, 0, 0};
    int k0 = 0;
    for (; k0 + 16 <= K; k0 += 16) {
      double a[4], b[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * s + q;
        a[s] = TA ? A[k * lda + m] : A[m * lda + k];
        b[s] = TB ? B[n * ldb + k] : B[k * ldb + n];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc[s], 0, 0, 0);
    }
    for (; k0 < K; k0 += 4) {
      const int k = k0 + q, kc = min(k, K - 1);
      double a = TA ? A[kc * lda + m] : A[m * lda + kc];
      double b = TB ? B[n * ldb + kc] : B[kc * ldb + n];
      a = k < K ? a : 0.0;
      b = k < K ? b : 0.0;
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[0], 0, 0, 0);
    }
    const ldsmm_d4 sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = m0 + q + 4 * j, col = n0 + r;
      if (row < M && col < N) {
        double v = alpha * sum[j];
        if (beta != 0.0) v += beta * Cin[row * ldci + col];
        C[row * ldc + col] = v;
      }
    }
  }
}

}  // namespace
}  // namespace ttr
