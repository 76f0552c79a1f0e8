// Symmetric eigendecomposition for the truncation step.
//
// The truncation of the left-orthogonal RtO output (section 3.2, remark after
// Algorithm 5; the mirror of the truncation loop of Algorithm 2) needs, at each bond, the
// leading singular triplets of H(X_n).  With G = H(X_n) H(X_n)^T = U s^2 U^T:
//   H(X_n) <- s^-1 U^T H(X_n),   X_{n-1} <- X_{n-1} x_3 (U s),
// which is the SVD truncation written with the Gram matrix (equal to it in
// exact arithmetic; singular values below about 1e-7 of the largest are
// resolved only to FP64 rounding of the Gram).
//
// G (n <= 96) is diagonalised by cyclic two-sided Jacobi in one workgroup
// with G and the accumulated rotations V resident in LDS.  Each round applies
// n/2 disjoint rotations at once (round-robin pairing): phase A computes the
// rotation of every pair, phase B updates every 2x2 block
// G[{p_k,q_k}][{p_m,q_m}] <- J_k^T G J_m and V[:, {p_m,q_m}] <- V J_m, with
// J = [[c, s], [-s, c]] chosen so that the (p, q) entry vanishes.
#include "fastmath.h"
#include "jacobi.h"
#include "tt_internal.h"

namespace ttr {
namespace {

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(const double *Gin, double *lam,
                                                                 double *Uout, int n,
                                                                 int *info, const int *gate) {
  jacobi_eig_kernel_body(Gin, lam, Uout, n, info, gate);
}

template <typename T>
__global__ __launch_bounds__(256) void trunc_factors_kernel(const double *lam, const double *U,
                                                            int n, int k, T *P, T *S,
                                                            double *tail, const int *gate) {
  trunc_factors_kernel_body<T>(lam, U, n, k, P, S, tail, gate);
}

}  // namespace

int sym_eig(const double *G, double *lam, double *U, int64_t n, hipStream_t s, int *info,
            const int *gate) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "eigenproblem larger than the limit");
  const int np = (int)((n + 1) & ~1);
  const size_t lds = 2 * sizeof(double) * (size_t)np * (size_t)(np + 1);
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)jacobi_eig_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048));
    attr_set = true;
  }
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(kEigThreads), lds, s, G, lam, U, (int)n,
                     info, gate);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int trunc_factors(const double *lam, const double *U, int64_t n, int64_t k, T *P, T *S,
                  double *tail, hipStream_t s, const int *gate) {
  hipLaunchKernelGGL((trunc_factors_kernel<T>), dim3(1), dim3(256), 0, s, lam, U, (int)n, (int)k,
                     P, S, tail, gate);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template int trunc_factors<double>(const double *, const double *, int64_t, int64_t, double *,
                                   double *, double *, hipStream_t, const int *);
template int trunc_factors<float>(const double *, const double *, int64_t, int64_t, float *,
                                  float *, double *, hipStream_t, const int *);

}  // namespace ttr
