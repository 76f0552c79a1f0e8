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
#include <algorithm>

#include "fastmath.h"
#include "jacobi.h"
#include "tt_internal.h"

namespace ttr {
namespace {

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(const double *Gin, double *lam,
                                                                 double *Uout, int n,
                                                                 int *info, const int *gate,
                                                                 int relative) {
  jacobi_eig_kernel_body(Gin, lam, Uout, n, info, gate, relative != 0);
}

// many independent problems, one workgroup each (problem b at G + b sG,
// lam + b sl, U + b sU, order n[b])
constexpr int kEigBatchMax = 64;
struct EigBatchArgs {
  const double *G;
  double *lam, *U;
  int64_t sG, sl, sU;
  int n[kEigBatchMax];
  int relative;
};
__global__ __launch_bounds__(kEigThreads) void jacobi_eig_batch_kernel(EigBatchArgs a) {
  const int b = blockIdx.x;
  jacobi_eig_kernel_body(a.G + b * a.sG, a.lam + b * a.sl, a.U + b * a.sU, a.n[b], nullptr,
                         nullptr, a.relative != 0);
}

template <typename T>
__global__ __launch_bounds__(256) void trunc_factors_kernel(const double *lam, const double *U,
                                                            int n, int k, T *P, T *S,
                                                            double *tail, const int *gate) {
  trunc_factors_kernel_body<T>(lam, U, n, k, P, S, tail, gate);
}

}  // namespace

int sym_eig(const double *G, double *lam, double *U, int64_t n, hipStream_t s, int *info,
            const int *gate, bool relative) {
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
                     info, gate, relative ? 1 : 0);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int sym_eig_batch(const double *G, int64_t sG, double *lam, int64_t sl, double *U, int64_t sU,
                  const int *n, int count, bool relative, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)jacobi_eig_batch_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048));
    attr_set = true;
  }
  for (int b0 = 0; b0 < count; b0 += kEigBatchMax) {
    const int cnt = std::min(kEigBatchMax, count - b0);
    EigBatchArgs a;
    a.G = G + b0 * sG;
    a.lam = lam + b0 * sl;
    a.U = U + b0 * sU;
    a.sG = sG;
    a.sl = sl;
    a.sU = sU;
    a.relative = relative ? 1 : 0;
    int nmax = 1;
    for (int k = 0; k < kEigBatchMax; ++k) a.n[k] = 0;
    for (int k = 0; k < cnt; ++k) {
      if (n[b0 + k] < 1 || n[b0 + k] > TT_MAX_SKETCH_RANK)
        return fail(TT_EUNSUPPORTED, "eigenproblem order outside 1 .. TT_MAX_SKETCH_RANK");
      if ((int64_t)n[b0 + k] * n[b0 + k] > std::min(sG, sU) || n[b0 + k] > sl)
        return fail(TT_EINVAL, "internal: eigenproblem slot too small");
      a.n[k] = n[b0 + k];
      nmax = std::max(nmax, a.n[k]);
    }
    const int np = (nmax + 1) & ~1;
    const size_t lds = 2 * sizeof(double) * (size_t)np * (size_t)(np + 1);
    hipLaunchKernelGGL(jacobi_eig_batch_kernel, dim3(cnt), dim3(kEigThreads), lds, s, a);
    TTR_HIP(hipGetLastError());
  }
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
