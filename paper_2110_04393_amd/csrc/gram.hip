// Gram matrices of tall panels in FP64: G = A^T A for the thin QR of the
// sweep (Algorithm 5, CholeskyQR with an FP64 Gram) and G = H H^T for the
// truncation (the mirror of Algorithm 2's loop), n <= 128 columns.
//
// A workgroup takes a chunk of 32 or 64 rows of the panel (k), stages it in LDS
// as FP64 with one batch of loads (all in flight together), and forms the
// upper-triangle 16 x 16 blocks of the chunk's contribution with the f64
// MFMA, one block per wavefront at a time (sixteen wavefronts: the MFMA chain
// of a block is the latency to hide); each block is written with its mirror,
// so every split is a full n x n matrix.  The splits are added in a fixed order by the split sum of
// the GEMM module (bitwise reproducible), or written to G directly when the
// panel has one chunk.
#include <algorithm>

#include "tt_internal.h"

namespace ttr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

// panel rows per workgroup: 32, or 64 for panels of more than 256 x 32 rows
// (the split sum takes at most 256 splits)
constexpr int kGramThreads = 1024;  // sixteen wavefronts
constexpr int kMaxN = 128;
constexpr int kApplyGramMaxN = 96;  // chunk and R staged together in LDS

// A(k, m) of the panel: AKC = false: A is K x n row-major (leading dimension
// lda); AKC = true: the panel is stored transposed, n x K row-major (H of a
// core, rows of length lda).
template <typename TA, bool AKC, int kChunk>
__global__ __launch_bounds__(kGramThreads) void gram_kernel(const TA *A, int64_t lda, int n,
                                                            int64_t K, double *out, int direct,
                                                            int64_t ldg, const int *gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) double gs[];  // [kChunk][ld]
  const int ld = ((n + 15) / 16) * 16 + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * kChunk;
  const int nk = (int)min<int64_t>(kChunk, K - k0);
  const int np = ((n + 15) / 16) * 16;

  // stage rows k0 .. k0 + kChunk (zero beyond K and beyond n)
  constexpr int kPer = kChunk * kMaxN / kGramThreads;  // values per thread, at most
  const int total = kChunk * np;
  double v[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kGramThreads;
    int k, m;
    if (AKC) {  // consecutive threads along k (contiguous in memory)
      m = e / kChunk;
      k = e - m * kChunk;
    } else {  // consecutive threads along m
      k = e / np;
      m = e - k * np;
    }
    const bool ok = e < total && k < nk && m < n;
    v[t] = ok ? (double)(AKC ? A[(int64_t)m * lda + k0 + k] : A[(k0 + k) * lda + m]) : 0.0;
  }
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kGramThreads;
    if (e < total) {
      int k, m;
      if (AKC) {
        m = e / kChunk;
        k = e - m * kChunk;
      } else {
        k = e / np;
        m = e - k * np;
      }
      gs[k * ld + m] = v[t];
    }
  }
  __syncthreads();

  // upper-triangle blocks (I <= J) dealt round-robin to the wavefronts
  const int nb = np / 16, nblk = nb * (nb + 1) / 2;
  for (int blk = wave; blk < nblk; blk += kGramThreads / 64) {
    int I = 0, rem = blk;
    while (rem >= nb - I) {
      rem -= nb - I;
      ++I;
    }
    const int J = I + rem;
    d4_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const double *pa = gs + q * ld + 16 * I + r;
    const double *pb = gs + q * ld + 16 * J + r;
#pragma unroll 4
    for (int kk = 0; kk < kChunk; kk += 8) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk * ld], pb[kk * ld], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[(kk + 4) * ld], pb[(kk + 4) * ld], acc1,
                                                 0, 0, 0);
    }
    const d4_t acc = acc0 + acc1;
    // lane (r, q), register j: G(16 I + q + 4 j, 16 J + r)
    double *o = direct ? out : out + (int64_t)blockIdx.x * n * n;
    const int64_t ldo = direct ? ldg : n;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * I + q + 4 * j, col = 16 * J + r;
      if (row < n && col < n) {
        o[row * ldo + col] = acc[j];
        if (I != J) o[col * ldo + row] = acc[j];
      }
    }
  }
}

// Q = Y R for one chunk of rows of Y (K x n, row-major, FP64 or FP32
// storage) and the n x n upper-triangular FP64 R (the R^-1 of the previous
// CholeskyQR pass), in FP64 arithmetic, written to Q in the storage type,
// then the chunk's contribution to Q^T Q (of Q as stored) as in gram_kernel:
// the first
// CholeskyQR pass's product and the second pass's Gram in one launch, Q not
// read back.  The chunk and R are staged in LDS; the wavefronts form the
// chunk's 16 x 16 blocks of Q (k-steps past the block's last column skipped:
// R is zero below its diagonal; four accumulators over consecutive k-steps),
// the chunk of Q replaces that of Y in LDS, and the Gram follows.  Rows past
// K and columns past n are zero in both stagings, so they are zero in Q.
template <typename TS, int kChunk>
__global__ __launch_bounds__(kGramThreads) void apply_gram_kernel(const TS *Y, const double *R,
                                                                  TS *Q, int n, int64_t K,
                                                                  double *out, int direct,
                                                                  int64_t ldg, const int *gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __attribute__((aligned(16))) double gs[];  // [kChunk][ld], then R [np][ld]
  const int ld = ((n + 15) / 16) * 16 + 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * kChunk;
  const int nk = (int)min<int64_t>(kChunk, K - k0);
  const int np = ((n + 15) / 16) * 16;
  double *Rs = gs + kChunk * ld;
  for (int e = tid; e < kChunk * np; e += kGramThreads) {
    const int k = e / np, m = e - k * np;
    gs[k * ld + m] = (k < nk && m < n) ? (double)Y[(k0 + k) * n + m] : 0.0;
  }
  for (int e = tid; e < np * np; e += kGramThreads) {
    const int k = e / np, m = e - k * np;
    Rs[k * ld + m] = (k < n && m < n) ? R[k * n + m] : 0.0;
  }
  __syncthreads();
  // blocks of Q: at most (64 / 16) x (96 / 16) = 24, two per wavefront
  const int bm = kChunk / 16, bn = np / 16;
  d4_t acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int blk = wave + h * (kGramThreads / 64);
    if (blk < bm * bn) {
      const int I = blk / bn, J = blk - I * bn;
      const double *pa = gs + (16 * I + r) * ld + q;
      const double *pb = Rs + q * ld + 16 * J + r;
      const int kend = 16 * (J + 1);  // R(k, c) = 0 for k > c
      d4_t a4[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
      for (int kk = 0; kk < kend; kk += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          a4[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk + 4 * u], pb[(kk + 4 * u) * ld],
                                                      a4[u], 0, 0, 0);
      }
      acc[h] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
  }
  __syncthreads();  // every read of the chunk of Y is done
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int blk = wave + h * (kGramThreads / 64);
    if (blk < bm * bn) {
      const int I = blk / bn, J = blk - I * bn;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * I + q + 4 * j, col = 16 * J + r;
        const TS v = (TS)acc[h][j];
        gs[row * ld + col] = (double)v;
        if (row < nk && col < n) Q[(k0 + row) * n + col] = v;
      }
    }
  }
  __syncthreads();
  const int nb = np / 16, nblk = nb * (nb + 1) / 2;
  for (int blk = wave; blk < nblk; blk += kGramThreads / 64) {
    int Ib = 0, rem = blk;
    while (rem >= nb - Ib) {
      rem -= nb - Ib;
      ++Ib;
    }
    const int Jb = Ib + rem;
    d4_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const double *pa = gs + q * ld + 16 * Ib + r;
    const double *pb = gs + q * ld + 16 * Jb + r;
#pragma unroll 4
    for (int kk = 0; kk < kChunk; kk += 8) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk * ld], pb[kk * ld], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[(kk + 4) * ld], pb[(kk + 4) * ld], acc1,
                                                 0, 0, 0);
    }
    const d4_t g = acc0 + acc1;
    double *o = direct ? out : out + (int64_t)blockIdx.x * n * n;
    const int64_t ldo = direct ? ldg : n;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 16 * Ib + q + 4 * j, col = 16 * Jb + r;
      if (row < n && col < n) {
        o[row * ldo + col] = g[j];
        if (Ib != Jb) o[col * ldo + row] = g[j];
      }
    }
  }
}

int chunk_rows(int64_t K) { return (K + 31) / 32 <= 256 ? 32 : 64; }
int64_t chunks_of(int64_t K) { return (K + chunk_rows(K) - 1) / chunk_rows(K); }

template <typename TA, bool AKC, int kChunk>
int launch(const void *A, int64_t lda, int64_t n, int64_t K, double *G, int64_t ldg,
           void *partial, hipStream_t s, const int *gate) {
  const int64_t nc = (K + kChunk - 1) / kChunk;
  const int ld = (int)(((n + 15) / 16) * 16 + 2);
  const size_t lds = (size_t)kChunk * ld * sizeof(double);
  static bool attr = false;
  if (!attr && lds > 64 * 1024) {
    TTR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&gram_kernel<TA, AKC, kChunk>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr = true;
  }
  const bool direct = nc == 1;
  hipLaunchKernelGGL((gram_kernel<TA, AKC, kChunk>), dim3((unsigned)nc), dim3(kGramThreads), lds, s,
                     static_cast<const TA *>(A), lda, (int)n, K,
                     direct ? G : static_cast<double *>(partial), direct ? 1 : 0, ldg, gate);
  TTR_HIP(hipGetLastError());
  if (!direct) {
    GemmX g;  // the chunk splits, summed in a fixed order
    g.C = G;
    g.ldc = ldg;
    g.tc = DType::F64;
    g.M = n;
    g.N = n;
    g.K = 1;
    g.math = DType::F64;
    g.splits = (int)nc;
    g.partial = partial;
    g.gate = gate;
    TTR_TRY(gemm_reduce_splits(g, s));
  }
  return TT_OK;
}

template <typename TS, int kChunk>
int launch_apply(const TS *Y, const double *R, TS *Q, int64_t n, int64_t K, double *G,
                 int64_t ldg, void *partial, hipStream_t s, const int *gate) {
  const int64_t nc = (K + kChunk - 1) / kChunk;
  const int ld = (int)(((n + 15) / 16) * 16 + 2), np = (int)(((n + 15) / 16) * 16);
  const size_t lds = (size_t)(kChunk + np) * ld * sizeof(double);
  static bool attr = false;
  if (!attr) {
    TTR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&apply_gram_kernel<TS, kChunk>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr = true;
  }
  const bool direct = nc == 1;
  hipLaunchKernelGGL((apply_gram_kernel<TS, kChunk>), dim3((unsigned)nc), dim3(kGramThreads), lds, s,
                     Y, R, Q, (int)n, K, direct ? G : static_cast<double *>(partial),
                     direct ? 1 : 0, ldg, gate);
  TTR_HIP(hipGetLastError());
  if (!direct) {
    GemmX g;  // the chunk splits, summed in a fixed order
    g.C = G;
    g.ldc = ldg;
    g.tc = DType::F64;
    g.M = n;
    g.N = n;
    g.K = 1;
    g.math = DType::F64;
    g.splits = (int)nc;
    g.partial = partial;
    g.gate = gate;
    TTR_TRY(gemm_reduce_splits(g, s));
  }
  return TT_OK;
}

}  // namespace

static int g_gram_mode = 0;  // 0: this kernel where supported, 1: split-K GEMM

void gram_set_mode(int mode) { g_gram_mode = mode; }

bool gram_supported(int64_t n, int64_t K) {
  return n >= 1 && n <= kMaxN && K >= 1 && chunks_of(K) <= 256;
}

bool gram_enabled(int64_t n, int64_t K) { return g_gram_mode == 0 && gram_supported(n, K); }

size_t gram_partial_elems(int64_t n, int64_t K) {
  const int64_t nc = chunks_of(K);
  return nc > 1 ? (size_t)(nc * n * n) : 0;
}

bool apply_gram_supported(int64_t n, int64_t K) {
  return gram_enabled(n, K) && n <= kApplyGramMaxN;
}

int apply_gram_run(const void *Y, DType ts, const double *R, void *Q, int64_t n, int64_t K,
                   double *G, int64_t ldg, void *partial, size_t partial_bytes, hipStream_t s,
                   const int *gate) {
  if (!apply_gram_supported(n, K)) return fail(TT_EINVAL, "internal: fused product and Gram shape");
  if (gram_partial_elems(n, K) * sizeof(double) > partial_bytes)
    return fail(TT_EINVAL, "internal: split buffer too small for the Gram");
  const bool c32 = chunk_rows(K) == 32;
  if (ts == DType::F64) {
    const double *y = static_cast<const double *>(Y);
    double *q = static_cast<double *>(Q);
    return c32 ? launch_apply<double, 32>(y, R, q, n, K, G, ldg, partial, s, gate)
               : launch_apply<double, 64>(y, R, q, n, K, G, ldg, partial, s, gate);
  }
  if (ts == DType::F32) {
    const float *y = static_cast<const float *>(Y);
    float *q = static_cast<float *>(Q);
    return c32 ? launch_apply<float, 32>(y, R, q, n, K, G, ldg, partial, s, gate)
               : launch_apply<float, 64>(y, R, q, n, K, G, ldg, partial, s, gate);
  }
  return fail(TT_EINVAL, "internal: storage type of the fused product");
}

int gram_run(const void *A, DType ta, bool a_kc, int64_t lda, int64_t n, int64_t K, double *G,
             int64_t ldg, void *partial, size_t partial_bytes, hipStream_t s,
             const int *gate) {
  if (!gram_supported(n, K)) return fail(TT_EINVAL, "internal: Gram shape not supported");
  if (gram_partial_elems(n, K) * sizeof(double) > partial_bytes)
    return fail(TT_EINVAL, "internal: split buffer too small for the Gram");
  const bool c32 = chunk_rows(K) == 32;
  if (ta == DType::F64) {
    if (a_kc)
      return c32 ? launch<double, true, 32>(A, lda, n, K, G, ldg, partial, s, gate)
                 : launch<double, true, 64>(A, lda, n, K, G, ldg, partial, s, gate);
    return c32 ? launch<double, false, 32>(A, lda, n, K, G, ldg, partial, s, gate)
               : launch<double, false, 64>(A, lda, n, K, G, ldg, partial, s, gate);
  }
  if (ta == DType::F32) {
    if (a_kc)
      return c32 ? launch<float, true, 32>(A, lda, n, K, G, ldg, partial, s, gate)
                 : launch<float, true, 64>(A, lda, n, K, G, ldg, partial, s, gate);
    return c32 ? launch<float, false, 32>(A, lda, n, K, G, ldg, partial, s, gate)
               : launch<float, false, 64>(A, lda, n, K, G, ldg, partial, s, gate);
  }
  return fail(TT_EINVAL, "internal: Gram storage type");
}

}  // namespace ttr
