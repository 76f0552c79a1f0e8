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

// Upper Cholesky G = R^T R of the n x n FP64 matrix G (row-major,
// n <= NMAX), then Rinv = R^{-1} (upper triangular, row-major; with FP32
// storage also rounded to Rinv_f), by one workgroup of four wavefronts.
// With nsplit > 0, G is the sum (in index order) of nsplit split-K partial
// products part[p n^2 + e], so the Gram GEMM needs no reduction kernel.
//
// Lane c owns column c (and c + 64 when NMAX > 64); wavefront w owns the
// row block [w NMAX/4, (w+1) NMAX/4) of those columns, in registers.  Both
// factorisations are blocked by these row blocks:
// * Cholesky, block J = 0..3: wavefront J factorises its (already updated)
//   rows one pivot at a time, broadcasting values across its lanes with
//   readlane (no LDS, no barrier):
//     R[j][c] = A[j][c] / sqrt(d_j),  A[i][c] -= A[j][i] A[j][c] / d_j  (i in block J, i > j),
//   publishes the block rows of R to LDS, and after one barrier the
//   wavefronts below apply the block's rank-NMAX/4 update
//     A[i][c] -= sum_{j in J} R[j][i] R[j][c].
// * Inverse, block J = 3..0, right-looking on B = I:
//     X[j] = B[j] / R[j][j] (row j of R^{-1}),  B[i] -= R[i][j] X[j]  (i < j),
//   inside block J by its wavefront alone, then the block rows of X are
//   published and the wavefronts above subtract their contribution.
// Every loop is unrolled so that register indices are compile-time
// constants.  A pivot d_j that is not finite or not above 1e-14 of the
// original diagonal entry raises the flag (or_flag = 0: flag overwritten,
// else or-ed) and is replaced by the original diagonal (1 if that is not
// positive) so that the results stay finite.
constexpr int kCholThreads = 256;

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int NMAX>
__device__ __forceinline__ void chol_inv_kernel_body(const double *G, const double *part,
                                                                int nsplit, double *Rinv,
                                                                float *Rinv_f, int n, int *flag,
                                                                int or_flag) {
  constexpr int NC = (NMAX + 63) / 64;  // column slots per lane
  constexpr int RW = NMAX / 4;          // rows per wavefront (one block)
  static_assert(NMAX % 4 == 0, "rows split over four wavefronts");
  extern __shared__ double s_R[];       // NMAX x NMAX: G staging, then strict upper R
  __shared__ double s_X[RW * NC * 64];  // published block rows of R^{-1}
  __shared__ double s_d0[NMAX];
  __shared__ double s_rdi[NMAX];        // 1 / R[j][j]
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nn = (int64_t)n * n;
  // G (summing the split-K partials in index order) staged through LDS;
  // 16 elements per thread, two partials per round: 32 loads in flight
  if (tid == 0) s_bad = 0;
  for (int e0 = tid; e0 < n * n; e0 += 16 * kCholThreads) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = 0.0;
    if (nsplit > 0) {
      int p = 0;
      for (; p + 1 < nsplit; p += 2) {
        double w0[16], w1[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int e = min(e0 + k * kCholThreads, n * n - 1);
          w0[k] = part[p * nn + e];
          w1[k] = part[(p + 1) * nn + e];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = (v[k] + w0[k]) + w1[k];
      }
      if (p < nsplit) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] += part[p * nn + min(e0 + k * kCholThreads, n * n - 1)];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = G[min(e0 + k * kCholThreads, n * n - 1)];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = e0 + k * kCholThreads;
      if (e < n * n) s_R[e] = v[k];
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += kCholThreads) s_d0[i] = s_R[i * n + i];
  double a[NC][RW];
#pragma unroll
  for (int sl = 0; sl < NC; ++sl) {
    const int col = lane + 64 * sl;
    const int cc = min(col, n - 1);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int i = RW * wave + r;
      const double v = s_R[min(i, n - 1) * n + cc];
      a[sl][r] = (i < n && col < n) ? v : 0.0;
    }
  }
  __syncthreads();  // staging reads done before R overwrites it; s_d0 ready
  // ---- Cholesky
#pragma unroll
  for (int J = 0; J < 4; ++J) {
    if (RW * J < n) {
      if (wave == J) {
        int bad = 0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const int j = RW * J + r;
          if (j < n) {
            double d = lane_bcast(a[j / 64][r], j % 64);
            const double d0 = s_d0[j];
            if (!(d > 1e-14 * d0) || !(d0 > 0.0) || !isfinite(d)) {
              d = (d0 > 0.0 && isfinite(d0)) ? d0 : 1.0;
              bad = 1;
            }
            const double inv_r = rsq_f64(d);
            const double inv_d = inv_r * inv_r;
            double rv[NC], f[NC];
#pragma unroll
            for (int sl = 0; sl < NC; ++sl) {
              const int col = lane + 64 * sl;
              rv[sl] = a[sl][r];
              f[sl] = (col > j) ? rv[sl] * inv_d : 0.0;
              a[sl][r] = (col == j) ? d * inv_r : ((col > j) ? rv[sl] * inv_r : 0.0);
            }
#pragma unroll
            for (int r2 = 0; r2 < RW; ++r2) {
              if (r2 > r) {
                const int i = RW * J + r2;
                const double c = lane_bcast(rv[i / 64], i % 64);  // A[j][i]
#pragma unroll
                for (int sl = 0; sl < NC; ++sl) a[sl][r2] -= c * f[sl];
              }
            }
            if (lane == 0) s_rdi[j] = inv_r;
          }
        }
        if (bad && lane == 0) s_bad = 1;
        // block rows of R, strictly upper part
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const int j = RW * J + r;
#pragma unroll
          for (int sl = 0; sl < NC; ++sl) {
            const int col = lane + 64 * sl;
            if (col < NMAX) s_R[j * NMAX + col] = (col > j) ? a[sl][r] : 0.0;
          }
        }
      }
      __syncthreads();
      if (wave > J) {
        // A[i][c] -= sum_{j in J} R[j][i] R[j][c]; R[j][i] read per lane and
        // broadcast with readlane
        double rjc[RW][NC], rji[RW];
#pragma unroll
        for (int jj = 0; jj < RW; ++jj) {
          const int j = RW * J + jj;
#pragma unroll
          for (int sl = 0; sl < NC; ++sl) rjc[jj][sl] = s_R[j * NMAX + min(lane + 64 * sl, NMAX - 1)];
          rji[jj] = s_R[j * NMAX + RW * wave + (lane % RW)];
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
#pragma unroll
          for (int jj = 0; jj < RW; ++jj) {
            const double c = lane_bcast(rji[jj], r);  // R[j][RW wave + r]
#pragma unroll
            for (int sl = 0; sl < NC; ++sl) a[sl][r] -= c * rjc[jj][sl];
          }
        }
      }
    }
  }
  // ---- inverse: rows of B = I held like A's
#pragma unroll
  for (int sl = 0; sl < NC; ++sl)
#pragma unroll
    for (int r = 0; r < RW; ++r) a[sl][r] = (RW * wave + r == lane + 64 * sl) ? 1.0 : 0.0;
  __syncthreads();  // R and 1/R[j][j] complete
#pragma unroll
  for (int J = 3; J >= 0; --J) {
    if (RW * J < n) {
      if (wave == J) {
#pragma unroll
        for (int r = RW - 1; r >= 0; --r) {
          const int j = RW * J + r;
          if (j < n) {
            const double inv = s_rdi[j];
            double x[NC];
#pragma unroll
            for (int sl = 0; sl < NC; ++sl) {
              x[sl] = a[sl][r] * inv;
              a[sl][r] = x[sl];
            }
#pragma unroll
            for (int r2 = 0; r2 < RW; ++r2) {
              if (r2 < r) {
                const double rij = s_R[(RW * J + r2) * NMAX + j];  // R[i][j]
#pragma unroll
                for (int sl = 0; sl < NC; ++sl) a[sl][r2] -= rij * x[sl];
              }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int sl = 0; sl < NC; ++sl) s_X[r * (NC * 64) + lane + 64 * sl] = a[sl][r];
      }
      __syncthreads();
      if (wave < J) {
        // B[i][c] -= sum_{j in J} R[i][j] X[j][c]
        double xj[RW][NC];
#pragma unroll
        for (int jj = 0; jj < RW; ++jj)
#pragma unroll
          for (int sl = 0; sl < NC; ++sl) xj[jj][sl] = s_X[jj * (NC * 64) + lane + 64 * sl];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const double *rrow = s_R + (RW * wave + r) * NMAX + RW * J;
#pragma unroll
          for (int jj = 0; jj < RW; ++jj) {
            const double rij = rrow[jj];
#pragma unroll
            for (int sl = 0; sl < NC; ++sl) a[sl][r] -= rij * xj[jj][sl];
          }
        }
      }
      __syncthreads();  // s_X is rewritten by the next block
    }
  }
#pragma unroll
  for (int sl = 0; sl < NC; ++sl) {
    const int col = lane + 64 * sl;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int i = RW * wave + r;
      if (i < n && col < n) {
        const double x = (i <= col) ? a[sl][r] : 0.0;
        Rinv[(int64_t)i * n + col] = x;
        if (Rinv_f) Rinv_f[(int64_t)i * n + col] = (float)x;
      }
    }
  }
  if (tid == 0) {
    if (or_flag) {
      if (s_bad) *flag = 1;
    } else {
      *flag = s_bad;
    }
  }
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads) void chol_inv_kernel(const double *G, const double *part,
                                                                int nsplit, double *Rinv,
                                                                float *Rinv_f, int n, int *flag,
                                                                int or_flag) {
  chol_inv_kernel_body<NMAX>(G, part, nsplit, Rinv, Rinv_f, n, flag, or_flag);
}

// One workgroup Householder QR of the m x n row-major Y into Q (m x n), with
// `work` (m x n) as global scratch and `rdiag` (n) / `tau` (n) scratch.  Runs
// only if always != 0 or *flag != 0.  With use_lds the panel and Q live in
// LDS (2 m n doubles).  Columns are distributed over the wavefronts; each
// column's dot product is a wavefront reduction.
constexpr int kHhThreads = 1024;

template <typename T>
__device__ __forceinline__ void householder_kernel_body(const T *Y, T *Q, T *work_g,
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

template <typename T>
__global__ __launch_bounds__(kHhThreads) void householder_kernel(const T *Y, T *Q, T *work_g,
                                                                 double *rdiag, double *tau,
                                                                 int64_t m, int n,
                                                                 const int *flag, int always,
                                                                 int use_lds) {
  householder_kernel_body<T>(Y, Q, work_g, rdiag, tau, m, n, flag, always, use_lds);
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads) void chol_group_kernel(const CholGroupDesc *tab) {
  const CholGroupDesc &e = tab[blockIdx.x];
  chol_inv_kernel_body<NMAX>(e.G, nullptr, 0, e.Rinv, e.Rinv_f, e.n, e.flag, e.or_flag);
}

template <typename T>
__global__ __launch_bounds__(kHhThreads) void householder_group_kernel(const HhGroupDesc *tab) {
  const HhGroupDesc &e = tab[blockIdx.x];
  householder_kernel_body<T>(static_cast<const T *>(e.Y), static_cast<T *>(e.Q),
                             static_cast<T *>(e.work), e.rdiag, e.tau, e.m, e.n, e.flag, e.always,
                             e.use_lds);
}

}  // namespace

void qr_set_mode(int mode) { g_qr_mode = mode; }

size_t qr_partial_elems(int64_t m, int64_t n) {
  const int sp = gemm_pick_splits(n, n, m);
  return sp > 1 ? (size_t)sp * n * n : 0;
}

template <int NMAX>
static int chol_inv_launch(const double *G, const double *part, int nsplit, double *Rinv,
                           float *Rinv_f, int n, int *flag, int or_flag, hipStream_t s) {
  const size_t lds = sizeof(double) * NMAX * NMAX;
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)chol_inv_kernel<NMAX>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  hipLaunchKernelGGL((chol_inv_kernel<NMAX>), dim3(1), dim3(kCholThreads), lds, s, G, part, nsplit, Rinv,
                     Rinv_f, n, flag, or_flag);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

// Cholesky + inverse of the n x n Gram (n <= TT_MAX_SKETCH_RANK); nsplit > 0:
// the Gram is the sum of nsplit split-K partials in `part`.
static int chol_inv(const double *G, const double *part, int nsplit, double *Rinv, float *Rinv_f,
                    int n, int *flag, int or_flag, hipStream_t s) {
  if (n <= 32) return chol_inv_launch<32>(G, part, nsplit, Rinv, Rinv_f, n, flag, or_flag, s);
  if (n <= 64) return chol_inv_launch<64>(G, part, nsplit, Rinv, Rinv_f, n, flag, or_flag, s);
  if (n <= 96) return chol_inv_launch<96>(G, part, nsplit, Rinv, Rinv_f, n, flag, or_flag, s);
  return fail(TT_EUNSUPPORTED, "Cholesky of a Gram matrix wider than 96");
}

int chol_inverse(const double *G, int64_t n, double *Rinv, float *Rinv_f, int *flag,
                 hipStream_t s) {
  return chol_inv(G, nullptr, 0, Rinv, Rinv_f, (int)n, flag, 0, s);
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
    g.defer_reduce = true;  // the Cholesky kernel sums the partials
    TTR_TRY(gemmx_run(g, s));
    const int nsp = gemm_used_splits(g);
    TTR_TRY(chol_inv(ws.gram, (const double *)ws.partial, nsp > 1 ? nsp : 0, ws.rinv,
                     f32 ? ws.rinv_f : nullptr, (int)n, ws.flag, pass, s));
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

template <int NMAX>
static int chol_group_launch(const CholGroupDesc *d_tab, int count, hipStream_t s) {
  const size_t lds = sizeof(double) * NMAX * NMAX;
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)chol_group_kernel<NMAX>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  hipLaunchKernelGGL((chol_group_kernel<NMAX>), dim3(count), dim3(kCholThreads), lds, s, d_tab);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int chol_group_run(const CholGroupDesc *d_tab, int count, int nmax, hipStream_t s) {
  if (count <= 0) return TT_OK;
  if (nmax <= 32) return chol_group_launch<32>(d_tab, count, s);
  if (nmax <= 64) return chol_group_launch<64>(d_tab, count, s);
  if (nmax <= 96) return chol_group_launch<96>(d_tab, count, s);
  return fail(TT_EUNSUPPORTED, "Cholesky of a Gram matrix wider than 96");
}

size_t hh_group_desc(const void *Y, void *Q, int64_t m, int64_t n, QrScratch &ws, int always,
                     size_t elem, HhGroupDesc *d) {
  const bool lds = (m * n <= kHhLdsElems);
  d->Y = Y;
  d->Q = Q;
  d->work = ws.q1;
  d->rdiag = ws.rinv;
  d->tau = ws.rinv + n;
  d->m = m;
  d->n = (int)n;
  d->flag = ws.flag;
  d->always = always;
  d->use_lds = lds ? 1 : 0;
  return lds ? 2 * elem * (size_t)(m * n) : 0;
}

template <typename T>
int householder_group_run(const HhGroupDesc *d_tab, int count, size_t lds_bytes, hipStream_t s) {
  if (count <= 0) return TT_OK;
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)householder_group_kernel<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024));
    attr_set = true;
  }
  hipLaunchKernelGGL((householder_group_kernel<T>), dim3(count), dim3(kHhThreads), lds_bytes, s,
                     d_tab);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int householder_group_run<double>(const HhGroupDesc *, int, size_t, hipStream_t);
template int householder_group_run<float>(const HhGroupDesc *, int, size_t, hipStream_t);

}  // namespace ttr
