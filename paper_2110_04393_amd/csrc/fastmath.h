// FP64 reciprocal and reciprocal square root for latency-bound scalar chains
// (pivots, rotation angles).  The hardware v_rcp_f64 / v_rsq_f64 estimates are
// refined by two Newton steps, which leaves at most a couple of ulps of error
// (checked against IEEE division and sqrt in the GPU tests).  The IEEE-exact
// sequences cost several dependent instructions more per call.
#pragma once
#include <hip/hip_runtime.h>

namespace ttr {

__device__ __forceinline__ double rcp_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

__device__ __forceinline__ double rsq_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// sqrt(x) for x > 0 as x * rsq(x)
__device__ __forceinline__ double sqrt_f64(double x) { return x * rsq_f64(x); }

}  // namespace ttr
