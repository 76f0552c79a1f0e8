// Second pass of the truncation for kept directions far below the largest
// singular value.
//
// The truncation of the left-orthogonal RtO output (section 3.2, remark after
// Algorithm 5; the mirror of the truncation loop of Algorithm 2) keeps, at
// each bond, the k leading singular directions of H = H(X_n) (l x cols).  The
// first pass diagonalises the FP64 Gram G = H H^T.  Its eigenvalues carry an
// absolute error of about u lambda_1, so a kept direction with lambda_j far
// below lambda_1 (a near-low-rank input whose weak directions are partly
// kept) is resolved only to that level: the split inside the weak group and
// the orthonormality of the new core rows are lost.  The paper's SVD of the
// core resolves them at the level of the singular values instead.
//
// When the smallest kept eigenvalue is below tau lambda_1, this pass
// recovers that accuracy with two more contractions of H:
//   1. U1 = [U_s | U_w]: U_s the w eigenvectors of the first pass above
//      tau lambda_1 (accurate, separated from the rest), U_w an orthonormal
//      basis of their complement (Householder QR of U_s, Q formed explicitly)
//      .................................................. trunc_basis_kernel
//   2. B = U1^T H (GEMM) and G2 = B B^T (FP64 Gram of B): the weak rows of B
//      are formed and multiplied at their own scale
//   3. eigenpairs of the weak block G2[w:, w:] (cyclic Jacobi, absolute
//      accuracy at the scale of that block), T = blockdiag(I_w, U2_{k-w})
//      (l x k), the Gram of the kept rows T^T B is T^T G2 T = L L^T
//      (Cholesky, which also removes the small strong-weak couplings), and
//      F = L^-1 T^T, P = U1 G2 F^T ................... trunc_solve_kernel
//   4. new core C = F B (orthonormal rows, GEMM) and X_{n-1} <- X_{n-1} P:
//      P C = U1 B B^T F^T F B is H projected onto the kept row space.
//      Kept directions at the rounding level of B (no information left in
//      them) get zero rows of F and columns of P, and the core receives
//      orthonormal rows orthogonal to the others in their place
//      ........................................... trunc_complete_kernel
// ctl[0] (1 = run this pass), ctl[1] = w and ctl[3] = the leading dimension
// of the first pass's eigenvector array are written by the first pass; every
// kernel here and the GEMMs of steps 2 and 4 return at once when ctl[0] = 0.
#include <algorithm>

#include "fastmath.h"
#include "jacobi.h"
#include "tt_internal.h"

namespace ttr {
namespace {

constexpr int kBasisThreads = 256;
constexpr int kRefMaxN = TT_MAX_SKETCH_RANK;

// U1 (n x n, row-major) = Q of the full Householder QR of U[:, :w] (U with
// leading dimension ctl[3]); Q's first w columns are +-U[:, :w].
__global__ __launch_bounds__(kBasisThreads) void trunc_basis_kernel(const double *U, int n,
                                                                    const int *ctl, double *U1) {
  if (ctl[0] == 0) return;
  const int w = ctl[1], ldu = ctl[3];
  // A (n x w, row stride kRefMaxN + 1): columns of U; reflector j below row j
  extern __shared__ double lds_basis[];
  auto A = [&](int i, int j) -> double & { return lds_basis[i * (kRefMaxN + 1) + j]; };
  __shared__ double s_tau[kRefMaxN], s_dot[kRefMaxN];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * w; e += blockDim.x) {
    const int i = e / w, j = e - i * w;
    A(i, j) = U[i * ldu + j];
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    // reflector H_j = I - tau v v^T with v = x - alpha e_j, x = A[j:, j]
    if (tid == 0) {
      double nrm2 = 0.0;
      for (int i = j; i < n; ++i) nrm2 += A(i, j) * A(i, j);
      const double x0 = A(j, j);
      const double nrm = sqrt(nrm2);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vv = nrm2 - x0 * x0 + v0 * v0;
      s_tau[j] = vv > 0.0 ? 2.0 / vv : 0.0;
      A(j, j) = v0;  // the reflector occupies column j from row j on
    }
    __syncthreads();
    // A[j:, c] -= tau v (v^T A[j:, c]) for the remaining columns
    for (int c = j + 1 + tid; c < w; c += blockDim.x) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += A(i, j) * A(i, c);
      s_dot[c] = d;
    }
    __syncthreads();
    for (int e = tid; e < (n - j) * (w - j - 1); e += blockDim.x) {
      const int i = j + e / (w - j - 1), c = j + 1 + e % (w - j - 1);
      A(i, c) -= s_tau[j] * A(i, j) * s_dot[c];
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{w-1} I, applied from the last reflector
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, c = e - i * n;
    U1[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = w - 1; j >= 0; --j) {
    for (int c = tid; c < n; c += blockDim.x) {
      double d = 0.0;
      for (int i = j; i < n; ++i) d += A(i, j) * U1[i * n + c];
      s_dot[c] = d;
    }
    __syncthreads();
    for (int e = tid; e < (n - j) * n; e += blockDim.x) {
      const int i = j + e / n, c = e % n;
      U1[i * n + c] -= s_tau[j] * A(i, j) * s_dot[c];
    }
    __syncthreads();
  }
}

// Steps 3 of the header.  scratch: gw (n*n), lam2 (n), U2 (n*n), M1 (n*k),
// Li (k*k), Q2 (n*k) doubles.  F (k x n) and P (n x k) are written in the
// storage type T.  Dynamic LDS: the Jacobi solve's, at least (k*(k+1)) doubles.
constexpr double kNullRel = 1e-26;

template <typename T>
__global__ __launch_bounds__(kEigThreads) void trunc_solve_kernel(const double *G2,
                                                                  const double *U1, int n, int k,
                                                                  int *ctl, int *nullmask,
                                                                  double *scratch, T *F, T *P) {
  if (ctl[0] == 0) return;
  extern __shared__ double lds[];
  const int w = ctl[1];
  const int nw = n - w;
  double *gw = scratch, *lam2 = gw + n * n, *U2 = lam2 + n, *M1 = U2 + n * n;
  double *Li = M1 + n * k, *Q2 = Li + k * k;
  const int tid = threadIdx.x;
  for (int e = tid; e < nw * nw; e += blockDim.x) {
    const int i = e / nw, j = e - i * nw;
    gw[e] = G2[(w + i) * n + w + j];
  }
  __syncthreads();
  jacobi_eig_kernel_body(gw, lam2, U2, nw, nullptr, nullptr, false);
  __syncthreads();
  // T(i, j) = delta_ij (j < w); U2(i - w, j - w) (j >= w, i >= w); else 0
  auto Tij = [&](int i, int j) -> double {
    if (j < w) return i == j ? 1.0 : 0.0;
    return i >= w ? U2[(i - w) * nw + (j - w)] : 0.0;
  };
  // M1 = G2 T (n x k)
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, j = e - i * k;
    double acc = 0.0;
    if (j < w) {
      acc = G2[i * n + j];
    } else {
      for (int m = w; m < n; ++m) acc += G2[i * n + m] * U2[(m - w) * nw + (j - w)];
    }
    M1[e] = acc;
  }
  __syncthreads();
  // Gt = T^T M1 (k x k) into LDS, ld k + 1
  const int ldl = k + 1;
  double *L = lds;
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int a = e / k, b = e - a * k;
    double acc = 0.0;
    if (a < w) {
      acc = M1[a * k + b];
    } else {
      for (int m = w; m < n; ++m) acc += U2[(m - w) * nw + (a - w)] * M1[m * k + b];
    }
    L[a * ldl + b] = acc;
  }
  __syncthreads();
  // symmetrise (the two triangles of T^T G2 T differ by rounding)
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int a = e / k, b = e - a * k;
    if (a > b) {
      const double v = 0.5 * (L[a * ldl + b] + L[b * ldl + a]);
      L[a * ldl + b] = v;
    }
  }
  __syncthreads();
  // Cholesky Gt = L L^T (lower triangle, column by column).  A kept weak
  // direction whose part orthogonal to the previous ones is at the rounding
  // level of B (pivot <= kNullRel max_i G2_ii, i.e. below about 1e-13 of the
  // largest singular value) carries no information: its row of F and column
  // of P are set to zero and trunc_complete_kernel gives the core an
  // orthonormal row in its place.
  __shared__ int s_null;
  __shared__ double s_gmax;
  if (tid == 0) {
    double gm = 0.0;
    for (int i = 0; i < n; ++i) gm = fmax(gm, G2[i * n + i]);
    s_gmax = gm;
    s_null = 0;
  }
  __syncthreads();
  const double dnull = kNullRel * s_gmax;
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = L[j * ldl + j];
      const bool null = !(d > dnull);
      if (null) ++s_null;
      nullmask[j] = null ? 1 : 0;
      L[j * ldl + j] = null ? 1e300 : sqrt(d);
    }
    __syncthreads();
    const double ljj = L[j * ldl + j];
    for (int i = j + 1 + tid; i < k; i += blockDim.x) L[i * ldl + j] /= ljj;
    __syncthreads();
    for (int e = tid; e < (k - j - 1) * (k - j - 1); e += blockDim.x) {
      const int i = j + 1 + e / (k - j - 1), c = j + 1 + e % (k - j - 1);
      if (c <= i) L[i * ldl + c] -= L[i * ldl + j] * L[c * ldl + j];
    }
    __syncthreads();
  }
  // Li = L^-1 (lower), one column per thread by forward substitution
  for (int c = tid; c < k; c += blockDim.x) {
    for (int i = 0; i < k; ++i) {
      double acc = (i == c) ? 1.0 : 0.0;
      for (int m = c; m < i; ++m) acc -= L[i * ldl + m] * Li[m * k + c];
      Li[i * k + c] = (i < c) ? 0.0 : acc / L[i * ldl + i];
    }
  }
  __syncthreads();
  // F = Li T^T (k x n);  Q2 = M1 Li^T (n x k) = G2 F^T
  for (int e = tid; e < k * n; e += blockDim.x) {
    const int a = e / n, i = e - a * n;
    double acc = 0.0;
    for (int b = 0; b <= a; ++b) acc += Li[a * k + b] * Tij(i, b);
    F[e] = nullmask[a] ? (T)0 : (T)acc;
  }
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, a = e - i * k;
    double acc = 0.0;
    for (int b = 0; b <= a; ++b) acc += M1[i * k + b] * Li[a * k + b];
    Q2[e] = acc;
  }
  __syncthreads();
  // P = U1 Q2 (n x k)
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, a = e - i * k;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += U1[i * n + m] * Q2[m * k + a];
    P[e] = nullmask[a] ? (T)0 : (T)acc;
  }
  if (tid == 0) ctl[2] = s_null;
}

// Null rows of the new core C (k x cols; nullmask[j] = 1, the row is zero)
// receive orthonormal rows orthogonal to the others: pseudo-random rows X
// (a SplitMix64 hash of row and column, uniform in [-1, 1)), projected twice
// on the orthogonal complement of C's rows (X <- X - (X C^T) C), then
// orthonormalised among themselves (Cholesky of X X^T).  X lives in xs
// (k x cols, storage T); sc holds 2 k^2 doubles.
__device__ __forceinline__ double hash_unit(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

constexpr int kCompThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kCompThreads) void trunc_complete_kernel(T *C, int k, int64_t cols,
                                                                      const int *ctl,
                                                                      const int *nullmask, T *xs,
                                                                      double *sc) {
  if (ctl[0] == 0 || ctl[2] == 0) return;
  __shared__ int s_rows[kRefMaxN];
  __shared__ int s_m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = kCompThreads / 64;
  if (tid == 0) {
    int m = 0;
    for (int j = 0; j < k; ++j)
      if (nullmask[j]) s_rows[m++] = j;
    s_m = m;
  }
  __syncthreads();
  const int m = s_m;
  double *coef = sc, *gx = sc + k * k;
  for (int64_t e = tid; e < (int64_t)m * cols; e += kCompThreads) {
    const int a = (int)(e / cols);
    const int64_t c = e - (int64_t)a * cols;
    xs[e] = (T)hash_unit(((uint64_t)s_rows[a] << 40) ^ (uint64_t)c);
  }
  __syncthreads();
  for (int round = 0; round < 2; ++round) {
    // coef(a, i) = X_a . C_i, one wavefront per pair
    for (int pr = wave; pr < m * k; pr += nwaves) {
      const int a = pr / k, i = pr - a * k;
      double acc = 0.0;
      for (int64_t c = lane; c < cols; c += 64)
        acc += (double)xs[(int64_t)a * cols + c] * (double)C[(int64_t)i * cols + c];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) coef[a * k + i] = acc;
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)m * cols; e += kCompThreads) {
      const int a = (int)(e / cols);
      const int64_t c = e - (int64_t)a * cols;
      double x = (double)xs[e];
      for (int i = 0; i < k; ++i) x -= coef[a * k + i] * (double)C[(int64_t)i * cols + c];
      xs[e] = (T)x;
    }
    __syncthreads();
  }
  // X X^T = L L^T, X <- L^-1 X, written into the null rows of C
  for (int pr = wave; pr < m * m; pr += nwaves) {
    const int a = pr / m, b = pr - a * m;
    double acc = 0.0;
    if (b <= a) {
      for (int64_t c = lane; c < cols; c += 64)
        acc += (double)xs[(int64_t)a * cols + c] * (double)xs[(int64_t)b * cols + c];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    }
    if (lane == 0 && b <= a) gx[a * m + b] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < m; ++j) {
      double d = gx[j * m + j];
      for (int p = 0; p < j; ++p) d -= gx[j * m + p] * gx[j * m + p];
      const double ljj = sqrt(fmax(d, 1e-300));
      gx[j * m + j] = ljj;
      for (int i = j + 1; i < m; ++i) {
        double v = gx[i * m + j];
        for (int p = 0; p < j; ++p) v -= gx[i * m + p] * gx[j * m + p];
        gx[i * m + j] = v / ljj;
      }
    }
    // invert in place into coef (lower triangular)
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) {
        double acc = (i == c) ? 1.0 : 0.0;
        for (int p = c; p < i; ++p) acc -= gx[i * m + p] * coef[p * m + c];
        coef[i * m + c] = (i < c) ? 0.0 : acc / gx[i * m + i];
      }
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)m * cols; e += kCompThreads) {
    const int a = (int)(e / cols);
    const int64_t c = e - (int64_t)a * cols;
    double x = 0.0;
    for (int b = 0; b <= a; ++b) x += coef[a * m + b] * (double)xs[(int64_t)b * cols + c];
    C[(int64_t)s_rows[a] * cols + c] = (T)x;
  }
}

// ctl of the first pass from descending eigenvalues lam (for the solver
// branch that has no split logic of its own); U's leading dimension is n
__global__ void trunc_ctl_kernel(const double *lam, int n, int k, double tau, int *ctl) {
  if (threadIdx.x != 0) return;
  int w = 0;
  const double thr = tau * lam[0];
  while (w < k && lam[w] >= thr) ++w;
  ctl[0] = (tau > 0.0 && w < k) ? 1 : 0;
  ctl[1] = w;
  ctl[2] = 0;
  ctl[3] = n;
}

}  // namespace

int trunc_refine_ctl(const double *lam, int64_t n, int64_t k, double tau, int *ctl,
                     hipStream_t s) {
  hipLaunchKernelGGL(trunc_ctl_kernel, dim3(1), dim3(64), 0, s, lam, (int)n, (int)k, tau, ctl);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

size_t trunc_refine_scratch(int64_t n, int64_t k) {
  return (size_t)(n * n + n + n * n + n * k + k * k + n * k);
}

int trunc_refine_basis(const double *U, int64_t n, const int *ctl, double *U1, hipStream_t s) {
  if (n > kRefMaxN) return fail(TT_EUNSUPPORTED, "refinement larger than the limit");
  const size_t lds = sizeof(double) * (size_t)n * (kRefMaxN + 1);
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)trunc_basis_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024));
    attr_set = true;
  }
  hipLaunchKernelGGL(trunc_basis_kernel, dim3(1), dim3(kBasisThreads), lds, s, U, (int)n, ctl,
                     U1);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int trunc_refine_solve(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                       int *nullmask, double *scratch, T *F, T *P, hipStream_t s) {
  if (n > kRefMaxN || k < 1 || k > n) return fail(TT_EINVAL, "internal: refinement shape");
  const int np = (int)((n + 1) & ~1);
  const size_t lds = std::max<size_t>(2 * sizeof(double) * (size_t)np * (size_t)(np + 1),
                                      sizeof(double) * (size_t)k * (size_t)(k + 1));
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)trunc_solve_kernel<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096));
    attr_set = true;
  }
  hipLaunchKernelGGL((trunc_solve_kernel<T>), dim3(1), dim3(kEigThreads), lds, s, G2, U1, (int)n,
                     (int)k, ctl, nullmask, scratch, F, P);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int trunc_refine_complete(T *C, int64_t k, int64_t cols, const int *ctl, const int *nullmask,
                          T *xs, double *scratch, hipStream_t s) {
  if (k > kRefMaxN) return fail(TT_EINVAL, "internal: completion shape");
  hipLaunchKernelGGL((trunc_complete_kernel<T>), dim3(1), dim3(kCompThreads), 0, s, C, (int)k,
                     cols, ctl, nullmask, xs, scratch);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int trunc_refine_complete<double>(double *, int64_t, int64_t, const int *, const int *,
                                           double *, double *, hipStream_t);
template int trunc_refine_complete<float>(float *, int64_t, int64_t, const int *, const int *,
                                          float *, double *, hipStream_t);

template int trunc_refine_solve<double>(const double *, const double *, int64_t, int64_t, int *,
                                        int *, double *, double *, double *, hipStream_t);
template int trunc_refine_solve<float>(const double *, const double *, int64_t, int64_t, int *,
                                       int *, double *, float *, float *, hipStream_t);

}  // namespace ttr
