// Dense contractions on the CDNA4 matrix cores (v_mfma_*_16x16x4).
//
// Every contraction of the method (partial contractions of Algorithm 3, the
// sketch product, projection and next-core product of Algorithm 5, Gram
// matrices) is C = alpha * A B + beta * C with A and B read through strides.
//
// Work decomposition.  A wavefront owns a (16 TM) x (16 TN) output tile made
// of 16x16 MFMA blocks; a workgroup is 4 wavefronts arranged WM x WN.  The K
// loop runs in chunks of 16: for MFMA step s (0..3) lane l = r + 16 q
// contributes A(m0 + r, k0 + 4q + s) and B(k0 + 4q + s, n0 + r).  Summing over
// s then covers k0 .. k0+15 exactly once; the permuted K order lets a lane
// read 4 consecutive K values of a K-contiguous operand from one cache line,
// and an M/N-contiguous operand is read by 16 lanes as one 128-byte line.
// Operands stream from HBM/L2 straight into registers: one f64 MFMA takes 64
// cycles per SIMD on gfx950, so 2 fragment loads per 4 MFMAs keep the matrix
// pipe fed without LDS staging.
//
// Output layout of a 16x16 block (MFMA D), lane l = r + 16 q, register j:
// column r; row q + 4 j for v_mfma_f64_16x16x4f64 (measured on gfx950) and
// 4 q + j for v_mfma_f32_16x16x4f32.
//
// Split-K: the K range is cut into chunks; each chunk writes its partial tile
// and a second kernel adds the chunks in index order, so results are bitwise
// reproducible (no float atomics).
#include "tt_internal.h"

namespace ttr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct AccOf;
template <>
struct AccOf<double> {
  typedef d4_t type;
};
template <>
struct AccOf<float> {
  typedef f4_t type;
};

// row of register j of lane group q in a 16x16 accumulator block
__device__ __forceinline__ int acc_row(double, int q, int j) { return q + 4 * j; }
__device__ __forceinline__ int acc_row(float, int q, int j) { return 4 * q + j; }

__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct TileMap {
  int64_t tiles_m, tiles_n, kchunk;
};

template <typename T, bool AKC, bool BKC, int TM, int TN, int WM, int WN>
__global__ __launch_bounds__(256) void gemm_kernel(Gemm<T> g, TileMap tm) {
  static_assert(WM * WN == 4, "4 wavefronts per workgroup");
  typedef typename AccOf<T>::type acc_t;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int wm = wave % WM, wn = wave / WM;
  int64_t wg = blockIdx.x;
  const int64_t tn_wg = wg % tm.tiles_n;
  wg /= tm.tiles_n;
  const int64_t tm_wg = wg % tm.tiles_m;
  wg /= tm.tiles_m;
  const int64_t split = (g.batch > 1) ? 0 : wg;
  const int64_t bidx = (g.batch > 1) ? wg : 0;
  const T *gA = g.A + bidx * g.sA;
  const T *gB = g.B + bidx * g.sB;
  T *gC = g.C + bidx * g.sC;

  const int64_t m0 = (tm_wg * WM + wm) * (16 * TM);
  const int64_t n0 = (tn_wg * WN + wn) * (16 * TN);
  if (m0 >= g.M || n0 >= g.N) return;  // no barriers below
  const int64_t kbeg = split * tm.kchunk;
  const int64_t kend = min(g.K, kbeg + tm.kchunk);
  const int r = lane & 15, q = lane >> 4;

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // per-lane base pointers at k = 4q
  const T *pa[TM];
  const T *pb[TN];
  bool rowok[TM], colok[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t m = m0 + 16 * i + r;
    rowok[i] = m < g.M;
    const int64_t mm = rowok[i] ? m : 0;
    pa[i] = AKC ? gA + mm * g.lda + 4 * q : gA + (int64_t)(4 * q) * g.lda + mm;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int64_t n = n0 + 16 * j + r;
    colok[j] = n < g.N;
    const int64_t nn = colok[j] ? n : 0;
    pb[j] = BKC ? gB + nn * g.ldb + 4 * q : gB + (int64_t)(4 * q) * g.ldb + nn;
  }

  for (int64_t k0 = kbeg; k0 < kend; k0 += 16) {
    T a[TM][4], b[TN][4];
    const bool kfull = (k0 + 16 <= kend);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * q + s;
      const bool kok = kfull || (k < kend);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const T *p = AKC ? pa[i] + k0 + s : pa[i] + (k0 + s) * g.lda;
        a[i][s] = (kok && rowok[i]) ? *p : T(0);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const T *p = BKC ? pb[j] + k0 + s : pb[j] + (k0 + s) * g.ldb;
        b[j][s] = (kok && colok[j]) ? *p : T(0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma(a[i][s], b[j][s], acc[i][j]);
  }

  // store
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + 16 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int64_t row = m0 + 16 * i + acc_row(T(0), q, jj);
        if (row >= g.M) continue;
        const T v = acc[i][j][jj];
        if (g.splits > 1) {
          g.partial[(split * g.M + row) * g.N + col] = v;
        } else {
          T *c = gC + row * g.ldc + col;
          *c = (g.beta != T(0)) ? g.alpha * v + g.beta * *c : g.alpha * v;
        }
      }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(Gemm<T> g) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = g.M * g.N;
  if (idx >= total) return;
  T s = 0;
  for (int p = 0; p < g.splits; ++p) s += g.partial[p * total + idx];
  const int64_t row = idx / g.N, col = idx - row * g.N;
  T *c = g.C + row * g.ldc + col;
  *c = (g.beta != T(0)) ? g.alpha * s + g.beta * *c : g.alpha * s;
}

struct Variant {
  int tm, tn, wm, wn;
};
constexpr Variant kVariants[] = {
    {1, 1, 1, 4},  // 16 x 64
    {1, 1, 4, 1},  // 64 x 16
    {1, 1, 2, 2},  // 32 x 32
    {2, 2, 2, 2},  // 64 x 64
};

int pick_variant(int64_t M, int64_t N) {
  // least padded work; ties go to the smaller tile (more workgroups)
  int best = 0;
  double best_cost = 1e300;
  for (int v = 0; v < 4; ++v) {
    const int64_t bm = 16 * kVariants[v].tm * kVariants[v].wm;
    const int64_t bn = 16 * kVariants[v].tn * kVariants[v].wn;
    const double cost = double((M + bm - 1) / bm * bm) * double((N + bn - 1) / bn * bn) *
                        (1.0 + 1e-3 * v);
    if (cost < best_cost) {
      best_cost = cost;
      best = v;
    }
  }
  return best;
}

template <typename T, bool AKC, bool BKC, int TM, int TN, int WM, int WN>
void launch_v(const Gemm<T> &g, const TileMap &tm, int64_t grid, hipStream_t s) {
  hipLaunchKernelGGL((gemm_kernel<T, AKC, BKC, TM, TN, WM, WN>), dim3((unsigned)grid), dim3(256),
                     0, s, g, tm);
}

template <typename T, bool AKC, bool BKC>
void launch_layout(int v, const Gemm<T> &g, const TileMap &tm, int64_t grid, hipStream_t s) {
  switch (v) {
    case 0: launch_v<T, AKC, BKC, 1, 1, 1, 4>(g, tm, grid, s); break;
    case 1: launch_v<T, AKC, BKC, 1, 1, 4, 1>(g, tm, grid, s); break;
    case 2: launch_v<T, AKC, BKC, 1, 1, 2, 2>(g, tm, grid, s); break;
    default: launch_v<T, AKC, BKC, 2, 2, 2, 2>(g, tm, grid, s); break;
  }
}

}  // namespace

int gemm_pick_splits(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const int v = pick_variant(M, N);
  const int64_t bm = 16 * kVariants[v].tm * kVariants[v].wm;
  const int64_t bn = 16 * kVariants[v].tn * kVariants[v].wn;
  const int64_t wgs = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  const int64_t want = 512;  // workgroups: 2 per CU
  if (wgs >= want / 2) return 1;
  int64_t sp = (want + wgs - 1) / wgs;
  const int64_t max_by_k = std::max<int64_t>(1, K / 128);  // >= 8 K-chunks each
  sp = std::min(sp, max_by_k);
  sp = std::min<int64_t>(sp, 256);
  return (int)std::max<int64_t>(1, sp);
}

template <typename T>
int gemm_run(const Gemm<T> &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return TT_OK;
  if (g.K <= 0) {
    return fail(TT_EINVAL, "gemm with K <= 0");
  }
  const int v = pick_variant(g.M, g.N);
  const int64_t bm = 16 * kVariants[v].tm * kVariants[v].wm;
  const int64_t bn = 16 * kVariants[v].tn * kVariants[v].wn;
  TileMap tm;
  tm.tiles_m = (g.M + bm - 1) / bm;
  tm.tiles_n = (g.N + bn - 1) / bn;
  if (g.batch > 1 && g.splits > 1) return fail(TT_EINVAL, "batched split-K gemm");
  if (g.batch < 1) return TT_OK;
  const int splits = std::max(1, g.splits);
  int64_t kchunk = (g.K + splits - 1) / splits;
  kchunk = (kchunk + 15) / 16 * 16;
  const int64_t used_splits = (g.K + kchunk - 1) / kchunk;
  Gemm<T> gg = g;
  gg.splits = (int)used_splits;
  tm.kchunk = kchunk;
  if (gg.splits > 1 && gg.partial == nullptr) return fail(TT_EINVAL, "split-K without buffer");
  const int64_t grid = tm.tiles_m * tm.tiles_n * (g.batch > 1 ? g.batch : used_splits);
  if (g.a_kc) {
    if (g.b_kc) launch_layout<T, true, true>(v, gg, tm, grid, s);
    else launch_layout<T, true, false>(v, gg, tm, grid, s);
  } else {
    if (g.b_kc) launch_layout<T, false, true>(v, gg, tm, grid, s);
    else launch_layout<T, false, false>(v, gg, tm, grid, s);
  }
  TTR_HIP(hipGetLastError());
  if (gg.splits > 1) {
    const int64_t total = g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, gg);
    TTR_HIP(hipGetLastError());
  }
  return TT_OK;
}

template int gemm_run<double>(const Gemm<double> &, hipStream_t);
template int gemm_run<float>(const Gemm<float> &, hipStream_t);

}  // namespace ttr
