// Small data-movement kernels: strided 2-D copies, dst = alpha src + beta dst
// (assembling the first core of a sum, N = 1 copies, gathering outputs).
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

}  // namespace

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
