// Small data-movement kernels: strided 2-D copies, dst = alpha src + beta dst
// (assembling the first core of a sum, N = 1 copies, gathering outputs), the
// power-of-two renormalisation of a partial contraction, and FP32 -> BF16
// rounding of a caller-given sketch.
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
__global__ __launch_bounds__(kScaleThreads) void scale_pow2_kernel(T *x, int64_t count) {
  __shared__ float s_max[kScaleThreads / 64];
  const int tid = threadIdx.x;
  float m = 0.f;
  for (int64_t e = tid; e < count; e += kScaleThreads) m = fmaxf(m, fabsf((float)x[e]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((tid & 63) == 0) s_max[tid >> 6] = m;
  __syncthreads();
  m = 0.f;
  for (int w = 0; w < kScaleThreads / 64; ++w) m = fmaxf(m, s_max[w]);
  if (!(m > 0.f) || !isfinite(m)) return;
  int ex = 0;
  frexpf(m, &ex);  // m = f 2^ex, f in [0.5, 1): floor(log2 m) = ex - 1
  const T f = (T)ldexp(1.0, 1 - ex);
  for (int64_t e = tid; e < count; e += kScaleThreads) x[e] *= f;
}

__global__ __launch_bounds__(256) void to_bf16_kernel(__bf16 *dst, const float *src,
                                                      int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = bf16_rne(src[e]);
}

}  // namespace

template <typename T>
int scale_pow2(T *x, int64_t count, hipStream_t s) {
  if (count <= 0) return TT_OK;
  hipLaunchKernelGGL((scale_pow2_kernel<T>), dim3(1), dim3(kScaleThreads), 0, s, x, count);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int scale_pow2<float>(float *, int64_t, hipStream_t);
template int scale_pow2<double>(double *, int64_t, hipStream_t);

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

}  // namespace ttr
