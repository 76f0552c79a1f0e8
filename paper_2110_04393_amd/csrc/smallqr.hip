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
#include "fastmath.h"
#include "tt_internal.h"

namespace ttr {
namespace {

int g_qr_mode = 0;  // 0 auto, 1 householder, 2 cholqr2

constexpr int kCholThreads = 512;
constexpr int kCholMaxOwn = 10;  // upper-triangle entries per thread: 96*97/2 <= 512*10

// One workgroup: upper Cholesky G = R^T R of the n x n matrix G (row-major,
// global, n <= 96), then Rinv = R^{-1} (upper triangular, row-major, global).
// Every thread owns a fixed set of upper-triangle positions (i, k), so a step
// is one pass over owned entries and one barrier:
//   Cholesky step j:  A[i][k] -= A[j][i] A[j][k] / d_j   (j < i <= k),
//                     R[j][k]  = A[j][k] / sqrt(d_j)      (k >= j),
//   inverse step j (j = n-1..0, B = I initially):
//                     B[i][c] -= R[i][j] B[j][c] / R[j][j] (i < j <= c),
// and R^{-1}[i][c] = B[i][c] / R[i][i].  A pivot d_j that is not finite or not
// above 1e-14 of the original diagonal entry raises the flag (or_flag = 0:
// flag overwritten, else or-ed) and is replaced by the original diagonal so
// that the results stay finite.
__global__ __launch_bounds__(kCholThreads) void chol_inv_kernel(const double *G, double *Rinv,
                                                                float *Rinv_f, int n, int *flag,
                                                                int or_flag) {
  extern __shared__ double lds[];
  const int ld = n | 1;          // odd stride: fewer LDS bank conflicts
  double *A = lds;               // n x ld, working matrix, later B
  double *R = lds + n * ld;      // n x ld
  __shared__ double s_d0[96];    // original diagonal (pivot test)
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, k = e - i * n;
    A[i * ld + k] = G[e];
    R[i * ld + k] = 0.0;
  }
  for (int j = tid; j < n; j += blockDim.x) s_d0[j] = G[j * n + j];
  if (tid == 0) s_bad = 0;
  // owned upper-triangle entries, enumerated row by row
  int own_i[kCholMaxOwn], own_k[kCholMaxOwn];
  int nown = 0;
  {
    const int tri = n * (n + 1) / 2;
    int i = 0, rowstart = 0;  // row i covers indices [rowstart, rowstart + n - i)
    for (int e = tid; e < tri && nown < kCholMaxOwn; e += blockDim.x) {
      while (e >= rowstart + (n - i)) {
        rowstart += n - i;
        ++i;
      }
      own_i[nown] = i;
      own_k[nown] = i + (e - rowstart);
      ++nown;
    }
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double d = A[j * ld + j];
    const double d0 = s_d0[j];
    const bool bad = !(d > 1e-14 * d0) || !(d0 > 0.0) || !isfinite(d);
    if (bad) d = (d0 > 0.0 && isfinite(d0)) ? d0 : 1.0;
    if (bad && tid == 0) s_bad = 1;
    const double inv_r = rsq_f64(d);
    const double inv_d = inv_r * inv_r;
#pragma unroll
    for (int t = 0; t < kCholMaxOwn; ++t) {
      if (t >= nown) break;
      const int i = own_i[t], k = own_k[t];
      if (i == j) {
        R[j * ld + k] = (k == j) ? d * inv_r : A[j * ld + k] * inv_r;
      } else if (i > j) {
        A[i * ld + k] -= A[j * ld + i] * A[j * ld + k] * inv_d;
      }
    }
    __syncthreads();
  }
  // B = I on the owned upper triangle (A is free now)
#pragma unroll
  for (int t = 0; t < kCholMaxOwn; ++t) {
    if (t >= nown) break;
    A[own_i[t] * ld + own_k[t]] = (own_i[t] == own_k[t]) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = n - 1; j >= 1; --j) {
    const double inv_rjj = rcp_f64(R[j * ld + j]);
#pragma unroll
    for (int t = 0; t < kCholMaxOwn; ++t) {
      if (t >= nown) break;
      const int i = own_i[t], c = own_k[t];
      if (i < j && c >= j) A[i * ld + c] -= R[i * ld + j] * A[j * ld + c] * inv_rjj;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, c = e - i * n;
    const double x = (c >= i) ? A[i * ld + c] * rcp_f64(R[i * ld + i]) : 0.0;
    Rinv[e] = x;
    if (Rinv_f) Rinv_f[e] = (float)x;
  }
  if (tid == 0) {
    if (or_flag) {
      if (s_bad) *flag = 1;
    } else {
      *flag = s_bad;
    }
  }
}

// One workgroup Householder QR of the m x n row-major Y into Q (m x n), with
// `work` (m x n) as global scratch and `rdiag` (n) / `tau` (n) scratch.  Runs
// only if always != 0 or *flag != 0.  With use_lds the panel and Q live in
// LDS (2 m n doubles).  Columns are distributed over the wavefronts; each
// column's dot product is a wavefront reduction.
constexpr int kHhThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kHhThreads) void householder_kernel(const T *Y, T *Q, T *work_g,
                                                                 double *rdiag, double *tau,
                                                                 int64_t m, int n,
                                                                 const int *flag, int always,
                                                                 int use_lds) {
  if (!always && *flag == 0) return;
  extern __shared__ double hh_lds[];
  T *work = use_lds ? reinterpret_cast<T *>(hh_lds) : work_g;
  T *Qw = use_lds ? reinterpret_cast<T *>(hh_lds) + m * n : Q;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  __shared__ double s_red[kHhThreads / 64];
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
    if (tid == 0) {
      rdiag[j] = beta;
      tau[j] = t;
    }
    __syncthreads();
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
    Qw[e] = (i == c) ? T(1) : T(0);
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      for (int c = j + wave; c < n; c += nw) {
        double w = 0.0;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          w += vi * (double)Qw[i * n + c];
        }
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
        w *= t;
        for (int64_t i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)work[i * n + j];
          Qw[i * n + c] = (T)((double)Qw[i * n + c] - vi * w);
        }
      }
    }
    __syncthreads();
  }
  // diag(R) >= 0
  for (int64_t e = tid; e < m * n; e += blockDim.x) {
    const int c = (int)(e % n);
    const T v = (rdiag[c] < 0.0) ? -Qw[e] : Qw[e];
    Q[e] = v;
  }
}

}  // namespace

void qr_set_mode(int mode) { g_qr_mode = mode; }

size_t qr_partial_elems(int64_t m, int64_t n) {
  const int sp = gemm_pick_splits(n, n, m);
  return sp > 1 ? (size_t)sp * n * n : 0;
}

static int chol_inv(const double *G, double *Rinv, float *Rinv_f, int n, int *flag, int or_flag,
                    hipStream_t s) {
  const size_t lds = 2 * sizeof(double) * (size_t)n * (size_t)(n | 1);
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)chol_inv_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024));
    attr_set = true;
  }
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kCholThreads), lds, s, G, Rinv, Rinv_f, n,
                     flag, or_flag);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

constexpr int64_t kHhLdsElems = 10000;  // 2 * m * n doubles must fit in LDS

template <typename T>
static int householder(const T *Y, T *Q, T *work, double *rdiag, double *tau, int64_t m,
                       int64_t n, const int *flag, int always, hipStream_t s) {
  const bool lds = (m * n <= kHhLdsElems);
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)householder_kernel<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024));
    attr_set = true;
  }
  const size_t bytes = lds ? 2 * sizeof(T) * (size_t)(m * n) : 0;
  hipLaunchKernelGGL((householder_kernel<T>), dim3(1), dim3(kHhThreads), bytes, s, Y, Q, work,
                     rdiag, tau, m, (int)n, flag, always, lds ? 1 : 0);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int qr_thin(const T *Y, T *Q, int64_t m, int64_t n, QrScratch &ws, hipStream_t s) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "QR panel wider than the limit");
  if (m < n) return fail(TT_EINVAL, "thin QR needs m >= n");
  const bool small = (m * n <= kHhLdsElems);
  const bool householder_only = (g_qr_mode == 1) || (g_qr_mode == 0 && small);
  // Householder scratch: rdiag = rinv[0..n), tau = rinv[n..2n) (rinv holds
  // max(n*n, 2n) doubles); work = q1.
  if (householder_only)
    return householder<T>(Y, Q, reinterpret_cast<T *>(ws.q1), ws.rinv, ws.rinv + n, m, n,
                          ws.flag, 1, s);
  const bool f32 = sizeof(T) == 4;
  T *q1 = reinterpret_cast<T *>(ws.q1);
  const T *rinv_t = f32 ? reinterpret_cast<const T *>(ws.rinv_f) : reinterpret_cast<const T *>(ws.rinv);
  for (int pass = 0; pass < 2; ++pass) {
    const T *src = pass == 0 ? Y : q1;
    T *dst = pass == 0 ? q1 : Q;
    GemmX g;  // G = src^T src, accumulated in FP64
    g.A = src;
    g.lda = n;
    g.a_kc = false;
    g.ta = DTypeOf<T>::value;
    g.B = src;
    g.ldb = n;
    g.b_kc = false;
    g.tb = DTypeOf<T>::value;
    g.C = ws.gram;
    g.ldc = n;
    g.tc = DType::F64;
    g.math = DType::F64;
    g.M = n;
    g.N = n;
    g.K = m;
    g.splits = gemm_pick_splits(n, n, m);
    g.partial = ws.partial;
    TTR_TRY(gemmx_run(g, s));
    TTR_TRY(chol_inv(ws.gram, ws.rinv, f32 ? ws.rinv_f : nullptr, (int)n, ws.flag, pass, s));
    Gemm<T> h;  // dst = src Rinv, in the storage precision
    h.A = src;
    h.lda = n;
    h.a_kc = true;
    h.B = rinv_t;
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
  return householder<T>(Y, Q, q1, ws.rinv, ws.rinv + n, m, n, ws.flag, 0, s);
}

template int qr_thin<double>(const double *, double *, int64_t, int64_t, QrScratch &,
                             hipStream_t);
template int qr_thin<float>(const float *, float *, int64_t, int64_t, QrScratch &, hipStream_t);

}  // namespace ttr
