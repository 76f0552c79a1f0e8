// Random Gaussian TT sketch (Definition 3.1) drawn on the device.
//
// The paper fixes only the distribution of the sketch cores (iid centred
// normals of variance 1/(l_{n-1} I_n l_n)).  The generator is counter based so
// that any element can be produced independently by any thread:
//   key_n   = mix(seed + (n + 1) * gamma)                 (core n, 0-based)
//   a, b    = mix(key_n + (2p + 1) * gamma), mix(key_n + (2p + 2) * gamma)
//   u1      = ((a >> 11) + 1) * 2^-53  in (0, 1]
//   u2      = (b >> 11) * 2^-53        in [0, 1)
//   z_{2p}  = sqrt(-2 ln u1) cos(2 pi u2),  z_{2p+1} = sqrt(-2 ln u1) sin(2 pi u2)
// i.e. the SplitMix64 stream of Steele, Lea and Flood (2014) evaluated at a
// counter, followed by the Box-Muller transform.  mix() is SplitMix64's output
// function; gamma = 0x9E3779B97F4A7C15.
#include "tt_internal.h"

namespace ttr {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kMaxCoresPerLaunch = 48;

struct SketchTable {
  int ncores;
  int dtype;
  int64_t pair_begin[kMaxCoresPerLaunch + 1];  // prefix sums of pair counts
  int64_t count[kMaxCoresPerLaunch];
  uint64_t key[kMaxCoresPerLaunch];
  double sqrt_count[kMaxCoresPerLaunch];
  void *ptr[kMaxCoresPerLaunch];
};

// blockIdx.y picks the core, so the table reads are uniform over the
// workgroup; blockIdx.x strides over that core's element pairs.
__global__ __launch_bounds__(256) void sketch_kernel(SketchTable t) {
  const int c = blockIdx.y;
  const int64_t pairs = t.pair_begin[c + 1] - t.pair_begin[c];
  const int64_t cnt = t.count[c];
  const uint64_t key = t.key[c];
  const double scale = t.sqrt_count[c];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t a = mix64(key + (uint64_t)(2 * p + 1) * kGamma);
    const uint64_t b = mix64(key + (uint64_t)(2 * p + 2) * kGamma);
    const double u1 = ((double)(a >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(b >> 11) * 0x1.0p-53;
    const double rad = sqrt(-2.0 * log(u1));
    const double th = 6.283185307179586 * u2;
    double sn, cs;
    sincos(th, &sn, &cs);
    const double z0 = rad * cs / scale, z1 = rad * sn / scale;
    const int64_t e = 2 * p;
    if (t.dtype == TT_F64) {
      double *o = static_cast<double *>(t.ptr[c]);
      o[e] = z0;
      if (e + 1 < cnt) o[e + 1] = z1;
    } else if (t.dtype == TT_F32) {
      float *o = static_cast<float *>(t.ptr[c]);
      o[e] = (float)z0;
      if (e + 1 < cnt) o[e + 1] = (float)z1;
    } else {  // BF16: rounded to FP32, then to BF16 (both to nearest even)
      __bf16 *o = static_cast<__bf16 *>(t.ptr[c]);
      o[e] = bf16_rne((float)z0);
      if (e + 1 < cnt) o[e + 1] = bf16_rne((float)z1);
    }
  }
}

}  // namespace

int sketch_generate(uint64_t seed, int N, const int64_t *dims, const int64_t *sr, int dtype,
                    void *const *cores, hipStream_t s) {
  for (int base = 0; base < N; base += kMaxCoresPerLaunch) {
    SketchTable t;
    t.ncores = std::min(kMaxCoresPerLaunch, N - base);
    t.dtype = dtype;
    t.pair_begin[0] = 0;
    for (int c = 0; c < t.ncores; ++c) {
      const int n = base + c;
      const int64_t cnt = sr[n] * dims[n] * sr[n + 1];
      t.count[c] = cnt;
      t.key[c] = mix64(seed + (uint64_t)(n + 1) * kGamma);
      t.sqrt_count[c] = sqrt((double)cnt);
      t.ptr[c] = cores[n];
      t.pair_begin[c + 1] = t.pair_begin[c] + (cnt + 1) / 2;
    }
    int64_t most = 0;
    for (int c = 0; c < t.ncores; ++c)
      most = std::max(most, t.pair_begin[c + 1] - t.pair_begin[c]);
    if (most == 0) continue;
    // About 4096 workgroups over the whole launch, each thread a few pairs.
    const int64_t cap = std::max<int64_t>(1, 4096 / t.ncores);
    const int64_t bx = std::min<int64_t>((most + 255) / 256, cap);
    hipLaunchKernelGGL(sketch_kernel, dim3((unsigned)bx, (unsigned)t.ncores), dim3(256), 0, s, t);
    TTR_HIP(hipGetLastError());
  }
  return TT_OK;
}

}  // namespace ttr
