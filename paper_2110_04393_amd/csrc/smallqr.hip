// Thin QR of tall-skinny sketches (Algorithm 5 / Algorithm 7: QR of Y_n).
//
// Fast path: CholeskyQR2 in FP64.  G = Y^T Y (MFMA, split-K), G = R^T R by a
// one-workgroup Cholesky that also forms R^{-1}, Q1 = Y R^{-1} (MFMA); the same
// again on Q1.  Both Cholesky factors have positive diagonals, so the final
// R = R2 R1 has diag(R) > 0, the normalisation the rest of the method uses.
//
// Robust path: Householder QR in one workgroup, used for small panels and,
// without a host round trip, whenever a Cholesky pivot falls below
// 1e-14 of its original diagonal entry (the sketch is numerically rank
// deficient, e.g. rounding A+A with a sketch wider than the rank).  The
// Cholesky kernels raise a device flag; the Householder kernel is always
// enqueued and returns at once unless the flag is set.  Householder columns are
// sign-normalised afterwards so that diag(R) >= 0 (zero counts as +).
#include "tt_internal.h"

namespace ttr {
namespace {

int g_qr_mode = 0;  // 0 auto, 1 householder, 2 cholqr2

constexpr int kCholThreads = 256;

// One workgroup: upper Cholesky of the n x n matrix G (row-major, global),
// G = R^T R, then Rinv = R^{-1} (upper triangular, row-major, global).
// flag: set to 1 (or_flag = 0: overwritten) if a pivot is not positive and
// well above rounding level.
__global__ __launch_bounds__(kCholThreads) void chol_inv_kernel(const double *G, double *Rinv,
                                                                int n, int *flag, int or_flag) {
  extern __shared__ double lds[];
  double *A = lds;              // n*n, becomes R (upper)
  double *X = lds + n * n;      // n*n, becomes R^{-1}
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int nn = n * n;
  for (int e = tid; e < nn; e += blockDim.x) {
    A[e] = G[e];
    X[e] = 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  // diag of the input for the relative pivot test, kept in X's diagonal slots
  // (X is written column by column afterwards)
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double d = A[j * n + j];
      const double d0 = G[j * n + j];
      if (!(d > 1e-14 * d0) || !(d0 > 0.0) || !isfinite(d)) {
        s_bad = 1;
        d = (d0 > 0.0 && isfinite(d0)) ? d0 : 1.0;
      }
      A[j * n + j] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / A[j * n + j];
    for (int k = j + 1 + tid; k < n; k += blockDim.x) A[j * n + k] *= inv;
    __syncthreads();
    // trailing update of the upper triangle: A[i][k] -= R[j][i] R[j][k], j < i <= k
    const int m = n - j - 1;
    for (int t = tid; t < m * m; t += blockDim.x) {
      const int a = t / m, b = t - a * m;
      if (b < a) continue;
      const int i = j + 1 + a, k = j + 1 + b;
      A[i * n + k] -= A[j * n + i] * A[j * n + k];
    }
    __syncthreads();
  }
  // R^{-1}: column c solves R x = e_c by back substitution (thread c)
  for (int c = tid; c < n; c += blockDim.x) {
    X[c * n + c] = 1.0 / A[c * n + c];
    for (int i = c - 1; i >= 0; --i) {
      double sacc = 0.0;
      for (int j = i + 1; j <= c; ++j) sacc += A[i * n + j] * X[j * n + c];
      X[i * n + c] = -sacc / A[i * n + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < nn; e += blockDim.x) Rinv[e] = X[e];
  if (tid == 0) {
    if (or_flag) {
      if (s_bad) *flag = 1;
    } else {
      *flag = s_bad;
    }
  }
}

// One workgroup Householder QR of the m x n row-major Y into Q (m x n), with
// `work` (m x n) as scratch and `rdiag` (n) / `tau` (n) scratch.  Runs only if
// always != 0 or *flag != 0.  Columns are distributed over the 4 wavefronts;
// each column's dot product is a wavefront reduction.
template <typename T>
__global__ __launch_bounds__(256) void householder_kernel(const T *Y, T *Q, T *work, double *rdiag,
                                                          double *tau, int64_t m, int n,
                                                          const int *flag, int always) {
  if (!always && *flag == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  __shared__ double s_red[4];
  __shared__ double s_alpha, s_norm2;
  for (int64_t e = tid; e < m * n; e += blockDim.x) work[e] = Y[e];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // norm of the column below the diagonal, alpha = work[j][j]
    double acc = 0.0;
    for (int64_t i = j + 1 + tid; i < m; i += blockDim.x) {
      const double v = (double)work[i * n + j];
      acc += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s_red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
      double s2 = 0.0;
      for (int w = 0; w < nw; ++w) s2 += s_red[w];
      s_norm2 = s2;
      s_alpha = (double)work[(int64_t)j * n + j];
    }
    __syncthreads();
    const double alpha = s_alpha, sigma = s_norm2;
    double beta, t, scale;
    if (sigma == 0.0) {
      beta = alpha;
      t = 0.0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v = [1; x / (alpha - beta)] stored below the diagonal
    for (int64_t i = j + 1 + tid; i < m; i += blockDim.x)
      work[i * n + j] = (T)((double)work[i * n + j] * scale);
    __syncthreads();
    if (tid == 0) {
      rdiag[j] = beta;
      tau[j] = t;
    }
    // apply H = I - t v v^T to columns j+1..n-1 (one wavefront per column)
    if (t != 0.0) {
      for (int c = j + 1 + wave; c < n; c += nw) {
        double w = 0.0;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          w += vi * (double)work[i * n + c];
        }
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
        w *= t;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          work[i * n + c] = (T)((double)work[i * n + c] - vi * w);
        }
      }
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{n-1} [I; 0], accumulated backwards
  for (int64_t e = tid; e < m * n; e += blockDim.x) {
    const int64_t i = e / n, c = e - i * n;
    Q[e] = (i == c) ? T(1) : T(0);
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      for (int c = j + wave; c < n; c += nw) {
        double w = 0.0;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          w += vi * (double)Q[i * n + c];
        }
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
        w *= t;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          Q[i * n + c] = (T)((double)Q[i * n + c] - vi * w);
        }
      }
    }
    __syncthreads();
  }
  // diag(R) >= 0
  for (int64_t e = tid; e < m * n; e += blockDim.x) {
    const int c = (int)(e % n);
    if (rdiag[c] < 0.0) Q[e] = -Q[e];
  }
}

}  // namespace

void qr_set_mode(int mode) { g_qr_mode = mode; }

size_t qr_partial_elems(int64_t m, int64_t n) {
  const int sp = gemm_pick_splits(n, n, m);
  return sp > 1 ? (size_t)sp * n * n : 0;
}

static int chol_inv(const double *G, double *Rinv, int n, int *flag, int or_flag, hipStream_t s) {
  const size_t lds = 2 * sizeof(double) * (size_t)n * n;
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)chol_inv_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024));
    attr_set = true;
  }
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kCholThreads), lds, s, G, Rinv, n, flag,
                     or_flag);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int qr_thin(const T *Y, T *Q, int64_t m, int64_t n, QrScratch &ws, hipStream_t s) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "QR panel wider than the limit");
  if (m < n) return fail(TT_EINVAL, "thin QR needs m >= n");
  const bool small = (m * n <= 32768);
  const bool householder_only = (g_qr_mode == 1) || (g_qr_mode == 0 && small);
  // Householder scratch: rdiag = rinv[0..n), tau = rinv[n..2n) (rinv holds
  // max(n*n, 2n) doubles); work = q1.
  if (householder_only) {
    T *work = reinterpret_cast<T *>(ws.q1);
    hipLaunchKernelGGL((householder_kernel<T>), dim3(1), dim3(256), 0, s, Y, Q, work, ws.rinv,
                       ws.rinv + n, m, (int)n, (const int *)ws.flag, 1);
    TTR_HIP(hipGetLastError());
    return TT_OK;
  }
  static_assert(sizeof(T) == 8, "CholeskyQR2 path is FP64 here");
  T *q1 = reinterpret_cast<T *>(ws.q1);
  T *partial = reinterpret_cast<T *>(ws.partial);
  for (int pass = 0; pass < 2; ++pass) {
    const T *src = pass == 0 ? Y : q1;
    T *dst = pass == 0 ? q1 : Q;
    Gemm<T> g;  // G = src^T src
    g.A = src;
    g.lda = n;
    g.a_kc = false;
    g.B = src;
    g.ldb = n;
    g.b_kc = false;
    g.C = ws.gram;
    g.ldc = n;
    g.M = n;
    g.N = n;
    g.K = m;
    g.splits = gemm_pick_splits(n, n, m);
    g.partial = partial;
    TTR_TRY(gemm_run<T>(g, s));
    TTR_TRY(chol_inv(ws.gram, ws.rinv, (int)n, ws.flag, pass, s));
    Gemm<T> h;  // dst = src Rinv
    h.A = src;
    h.lda = n;
    h.a_kc = true;
    h.B = ws.rinv;
    h.ldb = n;
    h.b_kc = false;
    h.C = dst;
    h.ldc = n;
    h.M = m;
    h.N = n;
    h.K = n;
    TTR_TRY(gemm_run<T>(h, s));
  }
  // fallback (no-op unless a pivot broke down); q1 and rinv are free again
  // once the GEMMs above have run (same stream).
  hipLaunchKernelGGL((householder_kernel<T>), dim3(1), dim3(256), 0, s, Y, Q, q1, ws.rinv,
                     ws.rinv + n, m, (int)n, (const int *)ws.flag, 0);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template int qr_thin<double>(const double *, double *, int64_t, int64_t, QrScratch &,
                             hipStream_t);

}  // namespace ttr
