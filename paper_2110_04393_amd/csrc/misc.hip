// Small data-movement kernels: strided 2-D copies, dst = alpha src + beta dst
// (assembling the first core of a sum, N = 1 copies, gathering outputs), the
// power-of-two renormalisation of a partial contraction, and FP32 -> BF16
// rounding of a caller-given sketch.
#include <algorithm>

#include "tt_internal.h"

namespace ttr {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void copy2d_kernel(T *dst, int64_t ldd, const T *src,
                                                     int64_t lds, int64_t rows, int64_t cols,
                                                     double alpha, double beta) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    const double v = alpha * (double)src[r * lds + c];
    dst[r * ldd + c] = (beta == 0.0) ? (T)v : (T)(v + beta * (double)dst[r * ldd + c]);
  }
}

// One workgroup: x <- x * 2^-e with e = floor(log2(max |x|)) (the maximum
// taken in FP32), so that the largest magnitude lands in [1/2, 2).
// Multiplying by a power of two is exact except for entries below 2^-126 of
// the largest, which become subnormal; the thin QR of Y_n = Z_n W_n is
// invariant under positive scalings of W_n (Q is unchanged, only R scales), so
// the rounding's output does not change.  Zero or non-finite maxima leave x
// untouched.
constexpr int kScaleThreads = 1024;

template <typename T>
__device__ __forceinline__ void scale_pow2_kernel_body(T *x, int64_t count,
                                                                   double *fout) {
  __shared__ float s_max[kScaleThreads / 64];
  const int tid = threadIdx.x;
  float m = 0.f;
  for (int64_t e = tid; e < count; e += kScaleThreads) m = fmaxf(m, fabsf((float)x[e]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((tid & 63) == 0) s_max[tid >> 6] = m;
  __syncthreads();
  m = 0.f;
  for (int w = 0; w < kScaleThreads / 64; ++w) m = fmaxf(m, s_max[w]);
  if (!(m > 0.f) || !isfinite(m)) {
    if (fout && tid == 0) *fout = 1.0;
    return;
  }
  int ex = 0;
  frexpf(m, &ex);  // m = f 2^ex, f in [0.5, 1): floor(log2 m) = ex - 1
  const T f = (T)ldexp(1.0, 1 - ex);
  for (int64_t e = tid; e < count; e += kScaleThreads) x[e] *= f;
  if (fout && tid == 0) *fout = (double)f;
}

template <typename T>
__global__ __launch_bounds__(kScaleThreads) void scale_pow2_kernel(T *x, int64_t count,
                                                                   double *fout) {
  scale_pow2_kernel_body<T>(x, count, fout);
}

// x *= *f (a factor that lives on the device)
template <typename T>
__global__ __launch_bounds__(256) void scale_dev_kernel(T *x, int64_t count, const double *f) {
  const T v = (T)*f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= v;
}

// C = tril(M) + tril(M, -1)^T for the k x k row-major M (symmetric copy of
// the lower triangle), scaled by alpha
template <typename T>
__global__ __launch_bounds__(256) void copyltu_kernel(T *C, const T *M, int64_t k, double alpha) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < k * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k, j = e - i * k;
    C[e] = (T)(alpha * (double)((i >= j) ? M[e] : M[j * k + i]));
  }
}

// Generalized Nystrom scalings from the eigenpairs (lam descending, U's
// columns the eigenvectors, row-major n x n) of G = C C^T: with s = sqrt(lam)
// the singular values of C, h_j = s_j^-1/2 for s_j > rcond s_1 (lam_j >
// rcond^2 lam_1) and 0 otherwise; A1 = U diag(h_j / s_j), A2 = diag(h) U^T.
__global__ __launch_bounds__(256) void nystrom_scale_kernel(const double *lam, const double *U,
                                                            int n, double rcond2, double *A1,
                                                            double *A2) {
  const double top = lam[0];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e - i * n;
    const double lj = lam[j], li = lam[i];
    const bool kj = top > 0.0 && lj > rcond2 * top, ki = top > 0.0 && li > rcond2 * top;
    const double hj = kj ? 1.0 / sqrt(sqrt(lj)) : 0.0;  // s_j^-1/2
    const double hi = ki ? 1.0 / sqrt(sqrt(li)) : 0.0;
    A1[e] = kj ? U[e] * (hj / sqrt(lj)) : 0.0;  // (i, j): U_ij h_j / s_j
    A2[e] = hi * U[j * n + i];                   // (i, j): h_i U_ji
  }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(__bf16 *dst, const float *src,
                                                      int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = bf16_rne(src[e]);
}

// dst (cols x rows) = src (rows x cols)^T, both row-major, 32 x 32 tiles
// through LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(T *dst, const T *src, int64_t rows,
                                                        int64_t cols) {
  __shared__ T tile[32][33];
  const int64_t tiles_c = (cols + 31) / 32;
  const int64_t r0 = (blockIdx.x / tiles_c) * 32, c0 = (blockIdx.x % tiles_c) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[c * rows + r] = tile[tx][k];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void identity_kernel(T *dst, int64_t m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m * m;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (e / m == e % m) ? T(1) : T(0);
}

// out = ||x||_F in FP64, one workgroup, fixed summation order.
template <typename T>
__global__ __launch_bounds__(256) void frob_kernel(const T *x, int64_t count, double *out) {
  __shared__ double s_part[4];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < count; e += 256) {
    const double v = (double)x[e];
    acc = fma(v, v, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = sqrt(((s_part[0] + s_part[1]) + s_part[2]) + s_part[3]);
}

// Rank of the eps-truncation: the smallest k >= 1 with
// sum_{j >= k} max(lam_j, 0) <= (eps0 * norm)^2 / (N - 1), capped by kmax;
// lam descending.  Also writes that tail.
__global__ void select_rank_kernel(const double *lam, int n, const double *norm, double eps0,
                                   int N, int kmax, int *k_out, double *tail_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double eps = eps0 * (*norm);
  const double thr = eps * eps / (double)(N - 1);
  double tail = 0.0;
  int k = n;
  for (int j = n - 1; j >= 1; --j) {  // tail after keeping j values
    const double t = tail + fmax(lam[j], 0.0);
    if (!(t <= thr)) break;
    tail = t;
    k = j;
  }
  if (k > kmax) {
    k = kmax;
    tail = 0.0;
    for (int j = k; j < n; ++j) tail += fmax(lam[j], 0.0);
  }
  *k_out = k;
  *tail_out = tail;
}

template <typename T>
__global__ __launch_bounds__(kScaleThreads) void scale_pow2_group_kernel(const ScaleGroupDesc *tab) {
  const ScaleGroupDesc &e = tab[blockIdx.x];
  scale_pow2_kernel_body<T>(static_cast<T *>(e.x), e.count, e.fout);
}

// X = R^{-1} of an upper-triangular n x n R (row-major, FP64), one column
// of X per thread by back substitution; Xf (optional) receives X rounded to
// FP32.  *flag = 1 (first = 1) or |= 1 when a diagonal entry is not above
// 64 u max_i |R_ii| or a result is not finite (R numerically singular).
__global__ __launch_bounds__(256) void tri_inv_upper_kernel(const double *R, int n, double *X,
                                                           float *Xf, int *flag, int first) {
  __shared__ double s_max;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid < 64) {  // one wavefront, its loads all in flight together
    double mx = 0.0;
    for (int i = tid; i < n; i += 64) mx = fmax(mx, fabs(R[i * n + i]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (tid == 0) {
      s_max = mx;
      s_bad = 0;
    }
  }
  __syncthreads();
  const double floor_d = 64.0 * 1.1102230246251565e-16 * s_max;
  for (int c = tid; c < n; c += blockDim.x) {
    bool bad = false;
    for (int i = n - 1; i >= 0; --i) {
      double v = 0.0;
      if (i <= c) {
        double acc = (i == c) ? 1.0 : 0.0;
        for (int m = i + 1; m <= c; ++m) acc -= R[i * n + m] * X[m * n + c];
        const double d = R[i * n + i];
        if (!(fabs(d) > floor_d)) bad = true;
        v = acc / d;
        if (!isfinite(v)) bad = true;
      }
      X[i * n + c] = v;
      if (Xf) Xf[i * n + c] = (float)v;
    }
    if (bad) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0) *flag = first ? s_bad : (*flag | s_bad);
}

// <X_j, Y> from the partial contraction W_1^(j) = H(X^(j)_{2:N}) H(Y_{2:N})^T:
// out[j] = sum_i X^(j)_1(i, :) W_1^(j) Y_1(i, :)^T (first cores 1 x I x r),
// one workgroup per j, fixed summation order.
template <typename T>
__global__ __launch_bounds__(256) void first_dots_kernel(FirstDots<T> a) {
  __shared__ double s_part[4];
  const int j = blockIdx.x;
  const T *X = a.X[j];
  const T *W = a.W[j];
  const int r = a.r[j];
  double acc = 0.0;
  for (int e = threadIdx.x; e < a.I * a.ry; e += 256) {
    const int i = e / a.ry, b = e - i * a.ry;
    double t = 0.0;
    for (int q = 0; q < r; ++q) t += (double)X[i * r + q] * (double)W[q * a.ry + b];
    acc += t * (double)a.Y[i * a.ry + b];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) a.out[j] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// Next core of a sum (sum_next_run): workgroup (summand j, a block of
// kSumNextI mode indices) stages the summand's columns of M once and each
// slice Y_j(:, i, :) in turn in LDS, and every thread forms outputs of the
// slice as dot products of length r_j.
constexpr int kSumNextThreads = 256, kSumNextI = 4;
constexpr size_t kSumNextLds = 64 * 1024;

struct SumNextArgs {
  const void *M;
  int64_t ldm;
  void *X;
  int64_t ldx, rs1, L, I1;
  const int *gate;
  int count;
  SumNextEntry e[kSumNextMax];
};

template <typename T>
__global__ __launch_bounds__(kSumNextThreads) void sum_next_kernel(SumNextArgs a) {
  if (a.gate && *a.gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char sn_lds[];
  T *As = reinterpret_cast<T *>(sn_lds);
  const int tid = threadIdx.x;
  const int64_t nib = (a.I1 + kSumNextI - 1) / kSumNextI;
  const int j = (int)(blockIdx.x / nib);
  const int64_t i0 = (int64_t)(blockIdx.x % nib) * kSumNextI;
  const SumNextEntry &e = a.e[j];
  const int L = (int)a.L, rj = e.rj, rj1 = e.rj1;
  T *Bs = As + L * rj;
  const T *M = static_cast<const T *>(a.M);
  const T *Y = static_cast<const T *>(e.Y);
  T *X = static_cast<T *>(a.X);
  for (int t = tid; t < L * rj; t += kSumNextThreads) {
    const int r = t / rj, c = t - r * rj;
    As[t] = M[r * a.ldm + e.offm + c];
  }
  const int64_t iend = min(i0 + kSumNextI, a.I1);
  for (int64_t i = i0; i < iend; ++i) {
    __syncthreads();  // the previous slice is no longer read
    for (int t = tid; t < rj * rj1; t += kSumNextThreads) {
      const int r = t / rj1, c = t - r * rj1;
      Bs[t] = Y[(r * a.I1 + i) * rj1 + c];
    }
    __syncthreads();
    for (int t = tid; t < L * rj1; t += kSumNextThreads) {
      const int r = t / rj1, c = t - r * rj1;
      T acc = T(0);
      for (int k = 0; k < rj; ++k) acc = fma(As[r * rj + k], Bs[k * rj1 + c], acc);
      X[r * a.ldx + i * a.rs1 + e.offn + c] = acc;
    }
  }
}

}  // namespace

template <typename T>
int transpose(T *dst, const T *src, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return TT_OK;
  const int64_t blocks = ((rows + 31) / 32) * ((cols + 31) / 32);
  hipLaunchKernelGGL((transpose_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, dst, src, rows,
                     cols);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int transpose<double>(double *, const double *, int64_t, int64_t, hipStream_t);
template int transpose<float>(float *, const float *, int64_t, int64_t, hipStream_t);

template <typename T>
int fill_identity(T *dst, int64_t m, hipStream_t s) {
  if (m <= 0) return TT_OK;
  const int64_t blocks = std::min<int64_t>((m * m + 255) / 256, 4096);
  hipLaunchKernelGGL((identity_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, dst, m);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int fill_identity<double>(double *, int64_t, hipStream_t);
template int fill_identity<float>(float *, int64_t, hipStream_t);

template <typename T>
int frob_norm(const T *x, int64_t count, double *out, hipStream_t s) {
  hipLaunchKernelGGL((frob_kernel<T>), dim3(1), dim3(256), 0, s, x, count, out);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int frob_norm<double>(const double *, int64_t, double *, hipStream_t);
template int frob_norm<float>(const float *, int64_t, double *, hipStream_t);

static size_t sum_next_lds(size_t elem, int64_t L, const SumNextEntry *e, int count) {
  size_t lds = 0;
  for (int j = 0; j < count; ++j)
    lds = std::max(lds, elem * (size_t)(L * e[j].rj + (int64_t)e[j].rj * e[j].rj1));
  return lds;
}

bool sum_next_fits(size_t elem, int64_t L, int64_t I1, const SumNextEntry *e, int count) {
  if (count < 1 || count > kSumNextMax || L < 1 || I1 < 1) return false;
  for (int j = 0; j < count; ++j)
    if (e[j].rj < 1 || e[j].rj1 < 1) return false;
  return sum_next_lds(elem, L, e, count) <= kSumNextLds;
}

template <typename T>
int sum_next_run(const T *M, int64_t ldm, T *X, int64_t L, int64_t I1, int64_t rs1,
                 const SumNextEntry *e, int count, const int *gate, hipStream_t s) {
  if (!sum_next_fits(sizeof(T), L, I1, e, count))
    return fail(TT_EINVAL, "internal: sum next-core shape");
  const size_t lds = sum_next_lds(sizeof(T), L, e, count);
  static bool attr = false;
  if (!attr && lds > 48 * 1024) {
    TTR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&sum_next_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSumNextLds));
    attr = true;
  }
  SumNextArgs a;
  a.M = M;
  a.ldm = ldm;
  a.X = X;
  a.ldx = I1 * rs1;
  a.rs1 = rs1;
  a.L = L;
  a.I1 = I1;
  a.gate = gate;
  a.count = count;
  for (int j = 0; j < count; ++j) a.e[j] = e[j];
  const int64_t nib = (I1 + kSumNextI - 1) / kSumNextI;
  hipLaunchKernelGGL(sum_next_kernel<T>, dim3((unsigned)(nib * count)), dim3(kSumNextThreads), lds,
                     s, a);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int sum_next_run<double>(const double *, int64_t, double *, int64_t, int64_t, int64_t,
                                  const SumNextEntry *, int, const int *, hipStream_t);
template int sum_next_run<float>(const float *, int64_t, float *, int64_t, int64_t, int64_t,
                                 const SumNextEntry *, int, const int *, hipStream_t);

int select_rank(const double *lam, int n, const double *norm, double eps0, int N, int kmax,
                int *k_out, double *tail_out, hipStream_t s) {
  hipLaunchKernelGGL(select_rank_kernel, dim3(1), dim3(64), 0, s, lam, n, norm, eps0, N, kmax,
                     k_out, tail_out);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int scale_pow2(T *x, int64_t count, hipStream_t s, double *fout) {
  if (count <= 0) return TT_OK;
  hipLaunchKernelGGL((scale_pow2_kernel<T>), dim3(1), dim3(kScaleThreads), 0, s, x, count, fout);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int scale_pow2<float>(float *, int64_t, hipStream_t, double *);
template int scale_pow2<double>(double *, int64_t, hipStream_t, double *);

template <typename T>
int scale_dev(T *x, int64_t count, const double *f, hipStream_t s) {
  if (count <= 0) return TT_OK;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL((scale_dev_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, x, count, f);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int scale_dev<float>(float *, int64_t, const double *, hipStream_t);
template int scale_dev<double>(double *, int64_t, const double *, hipStream_t);

template <typename T>
int copyltu(T *C, const T *M, int64_t k, double alpha, hipStream_t s) {
  if (k <= 0) return TT_OK;
  const int64_t blocks = std::min<int64_t>((k * k + 255) / 256, 4096);
  hipLaunchKernelGGL((copyltu_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, C, M, k, alpha);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int copyltu<float>(float *, const float *, int64_t, double, hipStream_t);
template int copyltu<double>(double *, const double *, int64_t, double, hipStream_t);

int nystrom_scale(const double *lam, const double *U, int64_t n, double rcond, double *A1,
                  double *A2, hipStream_t s) {
  if (n <= 0) return TT_OK;
  hipLaunchKernelGGL(nystrom_scale_kernel, dim3(1), dim3(256), 0, s, lam, U, (int)n,
                     rcond * rcond, A1, A2);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int tri_inv_upper(const double *R, int64_t n, double *X, float *Xf, int *flag, bool first,
                  hipStream_t s) {
  if (n <= 0) return TT_OK;
  hipLaunchKernelGGL(tri_inv_upper_kernel, dim3(1), dim3(256), 0, s, R, (int)n, X, Xf, flag,
                     first ? 1 : 0);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int first_dots(const FirstDots<T> &a, int count, hipStream_t s) {
  if (count <= 0) return TT_OK;
  if (count > kFirstDotsMax) return fail(TT_EINVAL, "internal: too many first-core dots");
  hipLaunchKernelGGL((first_dots_kernel<T>), dim3(count), dim3(256), 0, s, a);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int first_dots<double>(const FirstDots<double> &, int, hipStream_t);
template int first_dots<float>(const FirstDots<float> &, int, hipStream_t);

int round_to_bf16(__bf16 *dst, const float *src, int64_t count, hipStream_t s) {
  if (count <= 0) return TT_OK;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, count);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int copy2d(T *dst, int64_t ldd, const T *src, int64_t lds, int64_t rows, int64_t cols,
           double alpha, double beta, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return TT_OK;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL((copy2d_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, dst, ldd, src,
                     lds, rows, cols, alpha, beta);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template int copy2d<double>(double *, int64_t, const double *, int64_t, int64_t, int64_t, double,
                            double, hipStream_t);
template int copy2d<float>(float *, int64_t, const float *, int64_t, int64_t, int64_t, double,
                           double, hipStream_t);

template <typename T>
int scale_pow2_group(const ScaleGroupDesc *d_tab, int count, hipStream_t s) {
  if (count <= 0) return TT_OK;
  hipLaunchKernelGGL((scale_pow2_group_kernel<T>), dim3(count), dim3(kScaleThreads), 0, s, d_tab);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int scale_pow2_group<double>(const ScaleGroupDesc *, int, hipStream_t);
template int scale_pow2_group<float>(const ScaleGroupDesc *, int, hipStream_t);

}  // namespace ttr
