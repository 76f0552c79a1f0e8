// Thin QR of tall-skinny sketches (Algorithm 5 / Algorithm 7: QR of Y_n).
//
// Fast path: CholeskyQR2 in FP64.  G = Y^T Y (the panel-Gram kernel, MFMA over
// 32- or 64-row chunks and a split sum; the split-K GEMM for panels it does
// not take), G = R^T R by a one-workgroup Cholesky that also forms R^{-1},
// Q1 = Y R^{-1} (MFMA); the same again on Q1 (whose Gram is within rounding
// of I, so that its factor is usually taken to first order).  The product
// Q1 = Y R^{-1} (FP64 arithmetic, also with FP32 storage) and the Gram of Q1
// are one kernel (apply_gram_run, gram.hip).  Both Cholesky factors have positive
// diagonals, so the final R = R2 R1 has diag(R) > 0, the normalisation the
// rest of the method uses.
//
// Ill-conditioned panels: when a first-pass pivot falls below 1e-14 of its
// original diagonal entry, the same Cholesky kernel factors G + s I instead,
// s = 11 (m n + n (n + 1)) u trace(G) (shifted CholeskyQR, Fukaya et al.
// 2020), and sets flag bit 1; the second pass runs as usual and a third
// CholeskyQR pass restores orthogonality to rounding: the Gram kernel, the
// one-workgroup rescue kernel (the blocked Cholesky below with a stricter
// pivot test) and the GEMM Q R^-1 with a copy back, all gated on flag word 1,
// which the second pass sets when the first was shifted.
//
// Robust path: Householder QR in one workgroup, used for panels of at most 8
// columns and, without a host round trip, whenever a pivot still breaks down
// (flag bit 0: the sketch is rank deficient, e.g. rounding A+A with a sketch
// wider than the rank).  For the latter it runs inside the third pass's
// one-workgroup kernel (always enqueued, returning at once unless bit 0 or
// bit 1 is set).  Householder columns are sign-normalised
// afterwards so that diag(R) >= 0 (zero counts as +).
#include "fastmath.h"
#include <algorithm>

#include "cholblk.h"
#include "tt_internal.h"
#include "wave.h"

namespace ttr {
namespace {

int g_qr_mode = 0;  // 0 auto, 1 householder, 2 cholqr2

// Without shift_c: one factorisation as above.  With shift_c > 0 (first
// CholeskyQR pass): a breakdown is redone at once, in the same workgroup, on
// G + s I with s = shift_c trace(G) (the trace bounds ||Y||_2^2); the flag
// then reads 2 (bit 1: a third pass is due), or 3 if even the shifted matrix
// breaks down.  With go (speculative sweep): nothing runs once *go is 0, and
// a breakdown clears it instead of being repaired (the flag keeps it).
template <int NMAX>
__global__ __launch_bounds__(kCholThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void chol_inv_kernel(const double *G, double *Rinv,
                                                                float *Rinv_f, int n, int *flag,
                                                                int or_flag, double shift_c,
                                                                int *go) {
  if (go && *go == 0) return;
  const int bad = chol_inv_kernel_body<NMAX>(G, Rinv, Rinv_f, n, flag, or_flag);
  // second pass: word 1 = the third pass is due (the first pass was shifted
  // and nothing broke down since)
  if (or_flag && threadIdx.x == 0) flag[1] = ((flag[0] & 3) == 2) ? 1 : 0;
  if (!bad) return;
  if (go) {
    if (threadIdx.x == 0) *go = 0;
    return;
  }
  if (or_flag || !(shift_c > 0.0)) return;
  __shared__ double s_trace;
  if (threadIdx.x < 64) {  // one wavefront, its loads all in flight together
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) t += G[i * n + i];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (threadIdx.x == 0) s_trace = t;
  }
  __syncthreads();
  chol_inv_kernel_body<NMAX>(G, Rinv, Rinv_f, n, flag, 0, shift_c * s_trace, 2);
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
  if (!always && (*flag & 1) == 0) return;
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

// The one-workgroup part of the rescue after the second CholeskyQR pass.
// When the third pass is due (flag word 1, set by the second pass when the
// first one was shifted) it factors the Gram of Q (G3) by the blocked
// Cholesky with a pivot test of 1e-4 of the diagonal (cond(Q)^2 too large
// for one more pass to restore orthogonality to rounding fails it) into
// rinv; a failed pivot sets flag bit 0 and clears word 1.  Then, when bit 0
// is set (by the second pass, by the shifted first pass or by that
// Cholesky), Householder QR of Y into Q (word 1 cleared, so the gated GEMM
// and copy of the third pass do nothing).  Words read once at the start.
template <typename T, int NMAX>
__global__ __launch_bounds__(kHhThreads) void cholqr_rescue_kernel(const double *G3, double *rinv,
                                                                   float *rinv_f, int n,
                                                                   int *flag, const T *Y, T *Q,
                                                                   T *work_g, int64_t m,
                                                                   int use_lds) {
  const int fl = flag[0], due = flag[1];
  int hh = fl & 1;
  if (due) {
    // or_flag 0 with mark 2: flag word 0 reads 2 after it, 3 on a failed pivot
    if (chol_inv_kernel_body<NMAX, kHhThreads / 64>(G3, rinv, rinv_f, n, flag, 0, 0.0, 2, 1e-4))
      hh = 1;
  }
  if (!hh) return;
  __syncthreads();
  if (threadIdx.x == 0) flag[1] = 0;
  // rdiag = rinv[0..n), tau = rinv[n..2n)
  householder_kernel_body<T>(Y, Q, work_g, rinv, rinv + n, m, n, flag, 1, use_lds);
}

// dst = src for count elements when *gate != 0
template <typename T>
__global__ __launch_bounds__(256) void gated_copy_kernel(T *dst, const T *src, int64_t count,
                                                         const int *gate) {
  if (*gate == 0) return;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * 256)
    dst[e] = src[e];
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void chol_group_kernel(const CholGroupDesc *tab) {
  const CholGroupDesc &e = tab[blockIdx.x];
  chol_inv_kernel_body<NMAX>(e.G, e.Rinv, e.Rinv_f, e.n, e.flag, e.or_flag);
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
  // the Gram kernel's chunk splits or the split-K GEMM's partials, whichever
  // the Gram takes (both sizes, so that the choice can change between calls)
  const int sp = gemm_pick_splits(n, n, m, DType::F64);
  const size_t gemm_need = sp > 1 ? (size_t)sp * n * n : 0;
  return std::max(gemm_need, gram_supported(n, m) ? gram_partial_elems(n, m) : (size_t)0);
}

template <int NMAX>
static int chol_inv_launch(const double *G, double *Rinv, float *Rinv_f, int n, int *flag,
                           int or_flag, hipStream_t s, double shift_c, int *go) {
  hipLaunchKernelGGL((chol_inv_kernel<NMAX>), dim3(1), dim3(kCholThreads), 0, s, G, Rinv, Rinv_f,
                     n, flag, or_flag, shift_c, go);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

// Cholesky + inverse of the n x n Gram (n <= TT_MAX_SKETCH_RANK)
static int chol_inv(const double *G, double *Rinv, float *Rinv_f, int n, int *flag, int or_flag,
                    hipStream_t s, double shift_c = 0.0, int *go = nullptr) {
  if (n <= 32) return chol_inv_launch<32>(G, Rinv, Rinv_f, n, flag, or_flag, s, shift_c, go);
  if (n <= 64) return chol_inv_launch<64>(G, Rinv, Rinv_f, n, flag, or_flag, s, shift_c, go);
  if (n <= 96) return chol_inv_launch<96>(G, Rinv, Rinv_f, n, flag, or_flag, s, shift_c, go);
  return fail(TT_EUNSUPPORTED, "Cholesky of a Gram matrix wider than 96");
}

int chol_inverse(const double *G, int64_t n, double *Rinv, float *Rinv_f, int *flag,
                 hipStream_t s) {
  return chol_inv(G, Rinv, Rinv_f, (int)n, flag, 0, s);
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

// G = src^T src (n x n, FP64) by the Gram kernel, or the split-K GEMM where
// it does not apply; nothing runs while *gate is 0 (gate may be null)
template <typename T>
static int qr_gram(const T *src, int64_t m, int64_t n, QrScratch &ws, const int *gate,
                   hipStream_t s) {
  if (gram_enabled(n, m))
    return gram_run(src, DTypeOf<T>::value, false, n, n, m, ws.gram, n, ws.partial,
                    gram_partial_elems(n, m) * sizeof(double), s, gate);
  GemmX g;  // accumulated in FP64
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
  g.splits = gemm_pick_splits(n, n, m, DType::F64);
  g.partial = ws.partial;
  g.gate = gate;
  return gemmx_run(g, s);
}

// dst = src Rinv (m x n times the n x n R^-1, in the storage precision)
template <typename T>
static int qr_apply(const T *src, T *dst, int64_t m, int64_t n, const T *rinv, const int *gate,
                    hipStream_t s) {
  Gemm<T> h;
  h.A = src;
  h.lda = n;
  h.a_kc = true;
  h.B = rinv;
  h.ldb = n;
  h.b_kc = false;
  h.C = dst;
  h.ldc = n;
  h.M = m;
  h.N = n;
  h.K = n;
  GemmX hx = h.x();
  hx.gate = gate;
  return gemmx_run(hx, s);
}

template <typename T, int NMAX>
static int rescue_launch(const double *G3, double *rinv, float *rinv_f, int n, int *flag,
                         const T *Y, T *Q, T *q1, int64_t m, hipStream_t s) {
  // the Householder step keeps the panel in LDS when it fits beside the
  // kernel's static LDS (the Cholesky's panel buffers), else in q1
  static size_t max_dyn = 0;
  if (!max_dyn) {
    hipFuncAttributes fa;
    TTR_HIP(hipFuncGetAttributes(&fa, (const void *)cholqr_rescue_kernel<T, NMAX>));
    const size_t dyn = 160 * 1024 - fa.sharedSizeBytes;
    TTR_HIP(hipFuncSetAttribute((const void *)cholqr_rescue_kernel<T, NMAX>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    max_dyn = dyn;
  }
  const size_t need = 2 * sizeof(T) * (size_t)(m * n);
  const bool hh_lds = (m * n <= kHhLdsElems) && need <= max_dyn;
  const size_t lds = hh_lds ? need : 0;
  hipLaunchKernelGGL((cholqr_rescue_kernel<T, NMAX>), dim3(1), dim3(kHhThreads), lds, s, G3,
                     rinv, rinv_f, n, flag, Y, Q, q1, m, hh_lds ? 1 : 0);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

// The guarded rescue after the second CholeskyQR pass, all gated on the
// device (nothing runs on a panel that needs neither): the third pass, G3 =
// Q^T Q, its Cholesky and R3^-1, q1 = Q R3^-1 and Q <- q1 (gated on flag word
// 1), and the Householder fallback inside the rescue kernel (flag bit 0).
// q1 and rinv are free again once the second pass's GEMMs have run (same
// stream); q1 is also the Householder's global scratch when the panel does
// not fit in LDS.
template <typename T>
static int cholqr_fix(const T *Y, T *Q, T *q1, int64_t m, int64_t n, QrScratch &ws,
                      hipStream_t s) {
  if (n > 96) return fail(TT_EUNSUPPORTED, "QR panel wider than 96");
  const bool f32 = sizeof(T) == 4;
  int *const due = ws.flag + 1;
  TTR_TRY(qr_gram<T>(Q, m, n, ws, due, s));
  float *rf = f32 ? ws.rinv_f : nullptr;
  if (n <= 32) {
    TTR_TRY((rescue_launch<T, 32>(ws.gram, ws.rinv, rf, (int)n, ws.flag, Y, Q, q1, m, s)));
  } else if (n <= 64) {
    TTR_TRY((rescue_launch<T, 64>(ws.gram, ws.rinv, rf, (int)n, ws.flag, Y, Q, q1, m, s)));
  } else {
    TTR_TRY((rescue_launch<T, 96>(ws.gram, ws.rinv, rf, (int)n, ws.flag, Y, Q, q1, m, s)));
  }
  const T *rinv_t = f32 ? reinterpret_cast<const T *>(ws.rinv_f)
                        : reinterpret_cast<const T *>(ws.rinv);
  TTR_TRY(qr_apply<T>(Q, q1, m, n, rinv_t, due, s));
  const int64_t cnt = m * n;
  const unsigned blocks = (unsigned)std::min<int64_t>((cnt + 255) / 256, 1024);
  hipLaunchKernelGGL((gated_copy_kernel<T>), dim3(blocks), dim3(256), 0, s, Q, q1, cnt, due);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int qr_thin(const T *Y, T *Q, int64_t m, int64_t n, QrScratch &ws, hipStream_t s) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "QR panel wider than the limit");
  if (m < n) return fail(TT_EINVAL, "thin QR needs m >= n");
  const bool householder_only = (g_qr_mode == 1) || (g_qr_mode == 0 && n <= 8);
  // Householder scratch: rdiag = rinv[0..n), tau = rinv[n..2n) (rinv holds
  // max(n*n, 2n) doubles); work = q1.
  if (householder_only)
    return householder<T>(Y, Q, reinterpret_cast<T *>(ws.q1), ws.rinv, ws.rinv + n, m, n,
                          ws.flag, 1, s);
  const bool f32 = sizeof(T) == 4;
  T *q1 = reinterpret_cast<T *>(ws.q1);
  const T *rinv_t = f32 ? reinterpret_cast<const T *>(ws.rinv_f) : reinterpret_cast<const T *>(ws.rinv);
  // the first pass's product (FP64 arithmetic, Q1 rounded to the storage)
  // and the second pass's Gram in one launch
  const bool fused = apply_gram_supported(n, m);
  for (int pass = 0; pass < 2; ++pass) {
    const T *src = pass == 0 ? Y : q1;
    T *dst = pass == 0 ? q1 : Q;
    if (pass == 0 || !fused) TTR_TRY(qr_gram<T>(src, m, n, ws, ws.go, s));
    // first pass: shifted retry on breakdown, s = 11 (m n + n (n + 1)) u trace(G)
    // with u the unit roundoff of the storage (shifted CholeskyQR3)
    const double shift_c =
        pass == 0 ? 11.0 * (double)(m * n + n * (n + 1)) * (f32 ? 0x1p-24 : 0x1p-53) : 0.0;
    TTR_TRY(chol_inv(ws.gram, ws.rinv, f32 ? ws.rinv_f : nullptr, (int)n, ws.flag, pass, s,
                     shift_c, ws.go));
    if (pass == 0 && fused)
      TTR_TRY(apply_gram_run(src, DTypeOf<T>::value, ws.rinv, dst, n, m, ws.gram, n, ws.partial,
                             gram_partial_elems(n, m) * sizeof(double), s, ws.go));
    else
      TTR_TRY(qr_apply<T>(src, dst, m, n, rinv_t, ws.go, s));  // dst = src Rinv
  }
  // third pass when the first one was shifted and the Householder fallback
  // when a pivot broke down (no-ops otherwise).  The speculative form leaves
  // them out: its caller reads the flag back and redoes the QR guarded.
  if (ws.speculative) return TT_OK;
  return cholqr_fix<T>(Y, Q, q1, m, n, ws, s);
}

template int qr_thin<double>(const double *, double *, int64_t, int64_t, QrScratch &,
                             hipStream_t);
template int qr_thin<float>(const float *, float *, int64_t, int64_t, QrScratch &, hipStream_t);

template <int NMAX>
static int chol_group_launch(const CholGroupDesc *d_tab, int count, hipStream_t s) {
  hipLaunchKernelGGL((chol_group_kernel<NMAX>), dim3(count), dim3(kCholThreads), 0, s, d_tab);
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
