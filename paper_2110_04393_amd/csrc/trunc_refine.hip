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
//      basis of their complement (pivoted Cholesky of I - U_s U_s^T; built
//      by the first pass's finish kernel, tri_eig.hip)
//   2. B = U1^T H (GEMM) and G2 = B B^T (FP64 Gram of B): the weak rows of B
//      are formed and multiplied at their own scale
//   3. eigenpairs of the weak block G2[w:, w:] (cyclic Jacobi, absolute
//      accuracy at the scale of that block), T = blockdiag(I_w, U2_{k-w})
//      (l x k), the Gram of the kept rows T^T B is T^T G2 T = L L^T
//      (Cholesky, which also removes the small strong-weak couplings), and
//      F = L^-1 T^T, P = U1 G2 F^T ...... trunc_weak_kernel, trunc_final_kernel
//   4. new core C = F B (orthonormal rows, GEMM) and X_{n-1} <- X_{n-1} P:
//      P C = U1 B B^T F^T F B is H projected onto the kept row space.
//      Kept directions at the rounding level of B (no information left in
//      them) get zero rows of F and columns of P, and the core receives
//      orthonormal rows orthogonal to the others in their place
//      ............................. trunc_complete_prep/_rows_kernel
// ctl[0] (1 = run this pass), ctl[1] = w and ctl[3] = the leading dimension
// of the first pass's eigenvector array are written by the first pass; every
// kernel here and the GEMMs of steps 2 and 4 return at once when ctl[0] = 0.
#include <algorithm>

#include "cholblk.h"
#include "fastmath.h"
#include "jacobi.h"
#include "ldsmm.h"
#include "tt_internal.h"

namespace ttr {
namespace {

constexpr int kRefMaxN = TT_MAX_SKETCH_RANK;

// Step 3 of the header.  scratch: gw (n*n), lam2 (n), U2 (n*n), M1 (n*k),
// Q2 (n*k), R^-1 (k*k) doubles (trunc_refine_scratch).  F (k x n) and P
// (n x k) are written in the storage type T.
constexpr double kNullRel = 1e-26;

// Eigenpairs of the weak block G2[w:, w:] (lam2 descending, U2 columns),
// Jacobi in LDS.  scratch: gw (n*n), lam2 (n), U2 (n*n), M1 (n*k), Q2 (n*k).
__device__ void weak_block_eig(const double *G2, int n, int w, double *scratch) {
  const int nw = n - w;
  double *gw = scratch, *lam2 = gw + n * n, *U2 = lam2 + n;
  for (int e = threadIdx.x; e < nw * nw; e += blockDim.x) {
    const int i = e / nw, j = e - i * nw;
    gw[e] = G2[(w + i) * n + w + j];
  }
  __syncthreads();
  jacobi_eig_kernel_body(gw, lam2, U2, nw, nullptr, nullptr, false);
  __syncthreads();
}

// From the weak-block eigenvectors: T = blockdiag(I_w, U2[:, :k-w]), the
// Cholesky factor L of T^T G2 T (null directions detected), F = L^-1 T^T
// and P = U1 G2 F^T.  The products are f64 MFMA block products of the
// workgroup (lds_gemm); L^T and L^-T come from the blocked factorisation of
// the QR (cholblk.h) in its null mode, T^T G2 T staged in LDS.  scratch: gw
// (n*n, free again after the weak-block solve: F before its rounding), lam2
// (n), U2 (n*n), M1 (n*k, later P before its rounding), Q2 (n*k), R^-1
// (k*k).  Dynamic LDS: at least k*k doubles.
template <typename T, int NMAX>
__device__ void refine_factors(const double *G2, const double *U1, int n, int k, int *ctl,
                               int *nullmask, double *scratch, T *F, T *P) {
  extern __shared__ double lds[];
  const int w = ctl[1];
  const int nw = n - w, kw = k - w;
  double *Ft = scratch;
  double *U2 = scratch + n * n + n, *M1 = U2 + n * n;
  double *Q2 = M1 + n * k, *Ri = Q2 + n * k;
  double *Gt = lds;  // k x k
  const int tid = threadIdx.x;
  // M1 = G2 T: the first w columns are those of G2, the others G2[:, w:] U2[:, :k-w]
  for (int e = tid; e < n * w; e += blockDim.x) {
    const int i = e / w, j = e - i * w;
    M1[i * k + j] = G2[i * n + j];
  }
  if (kw > 0) lds_gemm<false, false>(G2 + w, n, U2, nw, M1 + w, k, n, kw, nw);
  __syncthreads();
  // Gt = T^T M1: the first w rows are those of M1, the others U2[:, :k-w]^T M1[w:, :]
  for (int e = tid; e < w * k; e += blockDim.x) Gt[e] = M1[e];
  if (kw > 0) lds_gemm<true, false>(U2, nw, M1 + w * k, k, Gt + w * k, k, kw, k, nw);
  __syncthreads();
  // symmetrise (the two triangles of T^T G2 T differ by rounding)
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int a = e / k, b = e - a * k;
    if (a > b) {
      const double v = 0.5 * (Gt[a * k + b] + Gt[b * k + a]);
      Gt[a * k + b] = v;
      Gt[b * k + a] = v;
    }
  }
  // A kept weak direction whose part orthogonal to the previous ones is at
  // the rounding level of B (pivot <= kNullRel max_i G2_ii, i.e. below about
  // 1e-13 of the largest singular value) carries no information: its row of
  // F and column of P are set to zero and trunc_complete_prep/_rows_kernel
  // give the core an orthonormal row in its place.
  __shared__ double s_gmax;
  if (tid < 64) {  // one wavefront, its loads all in flight together
    double gm = 0.0;
    for (int i = tid; i < n; i += 64) gm = fmax(gm, G2[i * n + i]);
    for (int off = 32; off > 0; off >>= 1) gm = fmax(gm, __shfl_xor(gm, off));
    if (tid == 0) s_gmax = gm;
  }
  __syncthreads();
  // Gt = R^T R, Ri = R^-1 (upper); L = R^T, L^-1 = Ri^T
  chol_inv_kernel_body<NMAX, kEigThreads / 64>(Gt, Ri, nullptr, k, nullptr, 0, 0.0, 0, 0.0,
                                               nullmask, kNullRel * s_gmax);
  // F = L^-1 T^T (k x n): columns < w are those of L^-1, the others
  // L^-1[:, w:k] U2[:, :k-w]^T = Ri[w:k, :]^T U2[:, :k-w]^T
  for (int e = tid; e < k * w; e += blockDim.x) {
    const int a = e / w, b = e - a * w;
    Ft[a * n + b] = Ri[b * k + a];
  }
  if (kw > 0) lds_gemm<true, true>(Ri + w * k, k, U2, nw, Ft + w, n, k, nw, kw);
  // Q2 = M1 L^-T = M1 Ri (n x k) = G2 T L^-T = G2 F^T
  lds_gemm<false, false>(M1, k, Ri, k, Q2, k, n, k, k);
  __syncthreads();
  for (int e = tid; e < k * n; e += blockDim.x) {
    const int a = e / n;
    F[e] = nullmask[a] ? (T)0 : (T)Ft[e];
  }
  // P = U1 Q2 (n x k), into M1
  lds_gemm<false, false>(U1, n, Q2, k, M1, k, n, k, n);
  __syncthreads();
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int a = e % k;
    P[e] = nullmask[a] ? (T)0 : (T)M1[e];
  }
  if (tid < 64) {
    int cnt = 0;
    for (int a = tid; a < k; a += 64) cnt += nullmask[a];
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (tid == 0) ctl[2] = cnt;
  }
}

// The weak eigenpairs (the factors follow in trunc_final_kernel, in
// tolerance mode once k is known).  With lamc: the spectrum the rank is
// chosen from, also when the second pass does not run; without: nothing
// runs unless it does.
__global__ __launch_bounds__(kEigThreads) void trunc_weak_kernel(const double *G2, int n,
                                                                 const int *ctl, double *scratch,
                                                                 const double *lam,
                                                                 double *lamc) {
  const int w = ctl[1];
  const bool second = ctl[0] != 0;
  if (!second && !lamc) return;
  if (second) weak_block_eig(G2, n, w, scratch);
  if (!lamc) return;
  // the spectrum the rank is chosen from: first-pass eigenvalues above the
  // split, second-pass ones below it
  const double *lam2 = scratch + n * n;
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    lamc[j] = (second && j >= w) ? lam2[j - w] : lam[j];
}

template <typename T, int NMAX>
__global__ __launch_bounds__(kEigThreads) void trunc_final_kernel(const double *G2,
                                                                  const double *U1, int n, int k,
                                                                  int *ctl, int *nullmask,
                                                                  double *scratch, T *F, T *P) {
  if (ctl[0] == 0) return;
  refine_factors<T, NMAX>(G2, U1, n, k, ctl, nullmask, scratch, F, P);
}

// Null rows of the new core C (k x cols, row-major; nullmask[j] = 1 marks a
// zero row) receive orthonormal rows orthogonal to the others.  The good
// rows are orthonormal, so for a unit vector e_i the residual
// r = e_i - C^T C e_i = e_i - sum_j C(j, i) C_j is orthogonal to them with
// no dot products to form, and |r|^2 = 1 - |C(:, i)|^2.  The first kernel
// (one workgroup) takes the m columns i of smallest |C(:, i)| (their squares
// sum to the number of good rows over cols >= k columns), forms the m x m
// Gram of the residuals, delta_ab - C(:, i_a) .
// C(:, i_b), its Cholesky factor L, and the coefficients W = L^-1 A,
// A(a, j) = C(j, i_a); the second writes row a of the completion
// sum_b L^-1(a, b) e_{i_b} - sum_j W(a, j) C_j, one column per thread.
// sc: trunc_complete_scratch(k, cols) doubles.
constexpr int kCompThreads = 1024;

template <typename T, int NMAX>
__global__ __launch_bounds__(kCompThreads) void trunc_complete_prep_kernel(
    const T *C, int k, int64_t cols, const int *ctl, const int *nullmask, double *sc) {
  if (ctl[0] == 0 || ctl[2] == 0) return;
  const int m = ctl[2];
  double *cn = sc;                        // cols: squared column norms of the good rows
  double *Li = cn + cols;                 // m x m
  double *W = Li + m * m;                 // m x k
  int *sel = reinterpret_cast<int *>(W + m * k);
  double *Ri = W + m * k + m;             // m x m: R^-1 of the residuals' Gram R^T R
  double *Gr = Ri + m * m;                // m x m: the residuals' Gram
  extern __shared__ double cp_lds[];
  double *Cs = cp_lds;                    // k x m: the selected columns (good rows)
  __shared__ int s_sel[kRefMaxN];
  const int tid = threadIdx.x;
  // squared column norms; a thread's columns c = tid + t kCompThreads stay
  // in registers for the selection when there are at most kPer of them
  constexpr int kPer = 8;
  const bool cached = cols <= (int64_t)kPer * kCompThreads;
  double mine[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) mine[t] = 1e300;
  for (int64_t c = tid; c < cols; c += kCompThreads) {
    double a = 0.0;
#pragma unroll 8
    for (int j = 0; j < k; ++j) {
      const double v = nullmask[j] ? 0.0 : (double)C[(int64_t)j * cols + c];
      a = fma(v, v, a);
    }
    if (cached) {
#pragma unroll
      for (int t = 0; t < kPer; ++t)
        if (c == tid + (int64_t)t * kCompThreads) mine[t] = a;
    } else {
      cn[c] = a;
    }
  }
  __syncthreads();
  // the m columns of smallest norm, one block-wide argmin per pick (ties to
  // the lower column)
  __shared__ double s_bv[kCompThreads / 64];
  __shared__ int64_t s_bi[kCompThreads / 64];
  const int lane = tid & 63, wave = tid >> 6;
  for (int a = 0; a < m; ++a) {
    double bv = 1e300;
    int64_t bi = cols;
    if (cached) {
#pragma unroll
      for (int t = 0; t < kPer; ++t)
        if (mine[t] < bv) {
          bv = mine[t];
          bi = tid + (int64_t)t * kCompThreads;
        }
    } else {
      for (int64_t c = tid; c < cols; c += kCompThreads)
        if (cn[c] < bv) {
          bv = cn[c];
          bi = c;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int64_t oi = __shfl_xor(bi, off);
      if (ov < bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_bv[wave] = bv;
      s_bi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w2 = 1; w2 < kCompThreads / 64; ++w2)
        if (s_bv[w2] < s_bv[0] || (s_bv[w2] == s_bv[0] && s_bi[w2] < s_bi[0])) {
          s_bv[0] = s_bv[w2];
          s_bi[0] = s_bi[w2];
        }
      s_sel[a] = (int)s_bi[0];
      if (!cached) cn[s_bi[0]] = 1e300;
    }
    __syncthreads();
    if (cached) {
      const int64_t cw = s_sel[a];
#pragma unroll
      for (int t = 0; t < kPer; ++t)
        if (cw == tid + (int64_t)t * kCompThreads) mine[t] = 1e300;
    }
  }
  // the selected columns over the good rows into LDS, then the residuals'
  // Gram delta_ab - C(:, i_a) . C(:, i_b)
  for (int e = tid; e < k * m; e += kCompThreads) {
    const int j = e / m, a = e - j * m;
    Cs[e] = nullmask[j] ? 0.0 : (double)C[(int64_t)j * cols + s_sel[a]];
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += kCompThreads) {
    const int a = e / m, b = e - a * m;
    double g = (a == b) ? 1.0 : 0.0;
    for (int j = 0; j < k; ++j) g = fma(-Cs[j * m + a], Cs[j * m + b], g);
    Gr[e] = g;
  }
  __syncthreads();
  // Gr = R^T R (blocked factorisation of the QR), L = R^T, L^-1 = Ri^T
  chol_inv_kernel_body<NMAX, kCompThreads / 64>(Gr, Ri, nullptr, m, nullptr, 0);
  for (int e = tid; e < m * m; e += kCompThreads) {
    const int i = e / m, c = e - i * m;
    Li[e] = Ri[c * m + i];
  }
  // W = L^-1 A, A(a, j) = C(j, sel_a) over the good rows
  for (int e = tid; e < m * k; e += kCompThreads) {
    const int a = e / k, j = e - a * k;
    double w = 0.0;
    for (int b = 0; b <= a; ++b) w = fma(Ri[b * m + a], Cs[j * m + b], w);
    W[e] = w;
  }
  for (int a = tid; a < m; a += kCompThreads) sel[a] = s_sel[a];
}


template <typename T>
__global__ __launch_bounds__(256) void trunc_complete_rows_kernel(T *C, int k, int64_t cols,
                                                                  const int *ctl,
                                                                  const int *nullmask,
                                                                  const double *sc) {
  if (ctl[0] == 0 || ctl[2] == 0) return;
  const int m = ctl[2];
  const double *Li = sc + cols, *W = Li + m * m;
  const int *sel = reinterpret_cast<const int *>(W + m * k);
  __shared__ int s_rows[kRefMaxN];
  if (threadIdx.x < 64) {  // the null rows in order, by ballots of 64 at a time
    const int lane = threadIdx.x;
    int base = 0;
    for (int j0 = 0; j0 < k; j0 += 64) {
      const int j = j0 + lane;
      const bool isnull = j < k && nullmask[j] != 0;
      const unsigned long long m = __ballot(isnull);
      if (isnull) s_rows[base + __popcll(m & ((1ull << lane) - 1))] = j;
      base += __popcll(m);
    }
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  // the column in registers (loops unrolled to the largest k)
  double col[kRefMaxN];
#pragma unroll
  for (int j = 0; j < kRefMaxN; ++j)
    col[j] = (j < k && !nullmask[j]) ? (double)C[(int64_t)j * cols + c] : 0.0;
  for (int a = 0; a < m; ++a) {
    double v = 0.0;
    for (int b = 0; b <= a; ++b)
      if (sel[b] == c) v += Li[a * m + b];
    const double *wa = W + a * k;
#pragma unroll
    for (int j = 0; j < kRefMaxN; ++j)
      if (j < k) v = fma(-wa[j], col[j], v);
    C[(int64_t)s_rows[a] * cols + c] = (T)v;
  }
}

// ctl of the first pass from descending eigenvalues lam and the full
// eigenvector matrix U (n x n) of the solver branch that has no split logic
// of its own; U1 = U (already a full orthonormal basis) when the second pass
// runs
__global__ void trunc_ctl_kernel(const double *lam, const double *U, int n, int k, double tau,
                                 int *ctl, double *U1) {
  __shared__ int s_second;
  if (threadIdx.x == 0) {
    int w = 0;
    const double thr = tau * lam[0];
    while (w < k && lam[w] >= thr) ++w;
    ctl[0] = (tau > 0.0 && w > 0 && w < k) ? 1 : 0;
    ctl[1] = w;
    ctl[2] = 0;
    ctl[3] = n;
    s_second = ctl[0];
  }
  __syncthreads();
  if (s_second)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) U1[e] = U[e];
}

__global__ void trunc_setk_kernel(int *ctl, int k) {
  if (threadIdx.x == 0) ctl[0] = (ctl[0] != 0 && k > ctl[1]) ? 1 : 0;
}

}  // namespace

int trunc_refine_setk(int *ctl, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(trunc_setk_kernel, dim3(1), dim3(64), 0, s, ctl, (int)k);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int trunc_refine_ctl(const double *lam, const double *U, int64_t n, int64_t k, double tau,
                     int *ctl, double *U1, hipStream_t s) {
  hipLaunchKernelGGL(trunc_ctl_kernel, dim3(1), dim3(256), 0, s, lam, U, (int)n, (int)k, tau, ctl,
                     U1);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

size_t trunc_refine_scratch(int64_t n, int64_t k) {
  return (size_t)(n * n + n + n * n + n * k + n * k + 2 * k * k);
}

template <typename T, int NMAX>
static int final_launch(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                        int *nullmask, double *scratch, T *F, T *P, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)k * (size_t)k;
  hipLaunchKernelGGL((trunc_final_kernel<T, NMAX>), dim3(1), dim3(kEigThreads), lds, s, G2, U1,
                     (int)n, (int)k, ctl, nullmask, scratch, F, P);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
static int final_run(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                     int *nullmask, double *scratch, T *F, T *P, hipStream_t s) {
  if (n > kRefMaxN || k < 1 || k > n) return fail(TT_EINVAL, "internal: refinement shape");
  if (k <= 32) return final_launch<T, 32>(G2, U1, n, k, ctl, nullmask, scratch, F, P, s);
  if (k <= 64) return final_launch<T, 64>(G2, U1, n, k, ctl, nullmask, scratch, F, P, s);
  return final_launch<T, 96>(G2, U1, n, k, ctl, nullmask, scratch, F, P, s);
}

static int weak_launch(const double *G2, int64_t n, int *ctl, double *scratch, const double *lam,
                       double *lamc, hipStream_t s) {
  const int np = (int)((n + 1) & ~1);
  const size_t lds = 2 * sizeof(double) * (size_t)np * (size_t)(np + 1);
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)trunc_weak_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096));
    attr_set = true;
  }
  hipLaunchKernelGGL(trunc_weak_kernel, dim3(1), dim3(kEigThreads), lds, s, G2, (int)n, ctl,
                     scratch, lam, lamc);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int trunc_refine_solve(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                       int *nullmask, double *scratch, T *F, T *P, hipStream_t s) {
  if (n > kRefMaxN || k < 1 || k > n) return fail(TT_EINVAL, "internal: refinement shape");
  TTR_TRY(weak_launch(G2, n, ctl, scratch, nullptr, nullptr, s));
  return final_run<T>(G2, U1, n, k, ctl, nullmask, scratch, F, P, s);
}

template <typename T>
int trunc_refine_complete(T *C, int64_t k, int64_t cols, const int *ctl, const int *nullmask,
                          double *scratch, hipStream_t s) {
  if (k > kRefMaxN || cols < k) return fail(TT_EINVAL, "internal: completion shape");
  // dynamic LDS: the selected columns (k x m, m <= k)
  const size_t lds = sizeof(double) * (size_t)(k * k);
  if (k <= 32)
    hipLaunchKernelGGL((trunc_complete_prep_kernel<T, 32>), dim3(1), dim3(kCompThreads), lds, s,
                       C, (int)k, cols, ctl, nullmask, scratch);
  else if (k <= 64)
    hipLaunchKernelGGL((trunc_complete_prep_kernel<T, 64>), dim3(1), dim3(kCompThreads), lds, s,
                       C, (int)k, cols, ctl, nullmask, scratch);
  else
    hipLaunchKernelGGL((trunc_complete_prep_kernel<T, 96>), dim3(1), dim3(kCompThreads), lds, s,
                       C, (int)k, cols, ctl, nullmask, scratch);
  TTR_HIP(hipGetLastError());
  hipLaunchKernelGGL((trunc_complete_rows_kernel<T>), dim3((unsigned)((cols + 255) / 256)),
                     dim3(256), 0, s, C, (int)k, cols, ctl, nullmask, scratch);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int trunc_refine_complete<double>(double *, int64_t, int64_t, const int *, const int *,
                                           double *, hipStream_t);
template int trunc_refine_complete<float>(float *, int64_t, int64_t, const int *, const int *,
                                          double *, hipStream_t);
size_t trunc_complete_scratch(int64_t k, int64_t cols) {
  // norms (cols), L^-1 (m*m), W (m*k), the picks (m ints), R^-1 and the
  // residuals' Gram (m*m each), m <= k
  return (size_t)(cols + 4 * k * k + 2 * k);
}

template <typename T>
int trunc_refine_eps(const double *G2, const double *U1, int64_t n, int *ctl, int *nullmask,
                     double *scratch, const double *lam, double *lamc, hipStream_t s) {
  (void)U1;
  (void)nullmask;
  return weak_launch(G2, n, ctl, scratch, lam, lamc, s);
}

template <typename T>
int trunc_refine_final(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                       int *nullmask, double *scratch, T *F, T *P, hipStream_t s) {
  return final_run<T>(G2, U1, n, k, ctl, nullmask, scratch, F, P, s);
}
template int trunc_refine_eps<double>(const double *, const double *, int64_t, int *, int *,
                                      double *, const double *, double *, hipStream_t);
template int trunc_refine_eps<float>(const double *, const double *, int64_t, int *, int *,
                                     double *, const double *, double *, hipStream_t);
template int trunc_refine_final<double>(const double *, const double *, int64_t, int64_t, int *,
                                        int *, double *, double *, double *, hipStream_t);
template int trunc_refine_final<float>(const double *, const double *, int64_t, int64_t, int *,
                                       int *, double *, float *, float *, hipStream_t);
template int trunc_refine_solve<double>(const double *, const double *, int64_t, int64_t, int *,
                                        int *, double *, double *, double *, hipStream_t);
template int trunc_refine_solve<float>(const double *, const double *, int64_t, int64_t, int *,
                                       int *, double *, float *, float *, hipStream_t);

}  // namespace ttr
