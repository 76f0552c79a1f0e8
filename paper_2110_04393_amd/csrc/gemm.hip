// Dense contractions on the CDNA4 matrix cores.
//
// Every contraction of the method (partial contractions of Algorithm 3, the
// sketch product, projection and next-core product of Algorithm 5, Gram
// matrices, truncation products) is C = alpha * A B + beta * C with A and B
// read through strides, in one of three arithmetic modes:
//   f64   v_mfma_f64_16x16x4f64
//   f32   v_mfma_f32_16x16x4f32
//   bf16  v_mfma_f32_16x16x32_bf16 (operands rounded to bf16 to nearest even,
//         fp32 accumulation)
// and with f64, f32 or bf16 storage of each operand (converted as the tiles
// are staged).
//
// Work decomposition.  A wavefront owns a (16 TM) x (16 TN) output tile made
// of 16x16 MFMA blocks; a workgroup is WM x WN wavefronts.  Operand tiles are
// staged through LDS (see the bodies below); lane l = r + 16 q supplies
// A(m0 + r, k) and B(k, n0 + r) for its k of the instruction: k0 + q for the
// x4 instructions (one value per MFMA), k0 + 8 q .. 8 q + 7 for bf16 (eight
// values packed into one MFMA).
//
// Accumulator layout of a 16x16 block, lane l = r + 16 q, register j:
// column r; row q + 4 j for the f64 instruction and 4 q + j for the f32 and
// bf16 ones (both measured on gfx950).
//
// Split-K: the K range is cut into chunks; each chunk writes its partial tile
// in the accumulator type and a second kernel adds the chunks in a fixed
// order (groups of eight in index order, then the group sums in index order),
// so results are bitwise reproducible (no float atomics).
#include "tt_internal.h"

namespace ttr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

struct MathF64 {
  typedef double in_t;
  typedef d4_t acc_t;
  typedef double part_t;
  static constexpr int CPL = 4;
  __device__ static int row(int q, int j) { return q + 4 * j; }
  __device__ static acc_t mma1(in_t a, in_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
struct MathF32 {
  typedef float in_t;
  typedef f4_t acc_t;
  typedef float part_t;
  static constexpr int CPL = 4;
  __device__ static int row(int q, int j) { return 4 * q + j; }
  __device__ static acc_t mma1(in_t a, in_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
struct MathBF16 {
  typedef float in_t;
  typedef f4_t acc_t;
  typedef float part_t;
  static constexpr int CPL = 8;
  __device__ static int row(int q, int j) { return 4 * q + j; }
};

template <typename To, typename From>
__device__ __forceinline__ To cvt(From v) {
  return (To)v;
}
template <>
__device__ __forceinline__ float cvt<float, __bf16>(__bf16 v) {
  return (float)v;
}
template <>
__device__ __forceinline__ double cvt<double, __bf16>(__bf16 v) {
  return (double)(float)v;
}

struct TileMap {
  int64_t tiles_m, tiles_n, kchunk;
};

constexpr int kSplitGroup = 8;

// Four consecutive elements from a 16-byte aligned address as vector loads,
// converted to the MFMA input type.
template <typename To>
__device__ __forceinline__ void load4(const double *p, To (&o)[4]) {
  typedef double d2_t __attribute__((ext_vector_type(2)));
  const d2_t x = *reinterpret_cast<const d2_t *>(p);
  const d2_t y = *reinterpret_cast<const d2_t *>(p + 2);
  o[0] = (To)x[0];
  o[1] = (To)x[1];
  o[2] = (To)y[0];
  o[3] = (To)y[1];
}
template <typename To>
__device__ __forceinline__ void load4(const float *p, To (&o)[4]) {
  const f4_t x = *reinterpret_cast<const f4_t *>(p);
  o[0] = (To)x[0];
  o[1] = (To)x[1];
  o[2] = (To)x[2];
  o[3] = (To)x[3];
}
template <typename To>
__device__ __forceinline__ void load4(const __bf16 *p, To (&o)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) o[s] = (To)(float)p[s];
}

// LDS-staged form for the x4 instructions (f64, f32).  The workgroup tile
// BM x BN = (16 TM WM) x (16 TN WN) (WM x WN wavefronts) advances over K in
// steps of BK (16 for the eight-wavefront tiles, 32 otherwise): all threads
// load the A (BM x BK) and B (BK x BN) tiles with coalesced reads (4
// consecutive elements of the contiguous dimension per thread), convert them
// to the MFMA type and store them k-major in LDS (As[k][m], Bs[k][n]); every
// wavefront then reads all its fragments of the step (A(m0 + r, k + q),
// B(k + q, n0 + r), lane = r + 16 q) before its MFMAs, so each operand
// element is fetched from memory once per workgroup.  The next tile is
// loaded into registers while the current one feeds the MFMAs (two LDS
// buffers, one barrier per step).  A row padding (8 doubles, 16 floats)
// spreads the four k-rows of a fragment read over the LDS banks.
//
// The f64 MFMA issues at about one instruction per 140 cycles from a single
// wavefront and needs several wavefronts per SIMD to approach its peak
// (measured on gfx950), so the tiles for outputs with a side of at most 64
// (most of the method's products) are 32 x 64 and 64 x 32 with eight
// 16 x 16 wavefronts: more workgroups and more wavefronts per CU.
template <int WM, int WN, int BKO>
constexpr int lds_bk() {
  return BKO ? BKO : (WM * WN == 8 ? 16 : 32);
}

template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN, int BKO>
__device__ __forceinline__ void gemm_lds_body(const GemmX &g, const TileMap &tm, int64_t wg) {
  static_assert(MT::CPL == 4, "x4 MFMA instructions");
  typedef typename MT::acc_t acc_t;
  typedef typename MT::in_t in_t;
  typedef typename MT::part_t part_t;
  constexpr int T = 64 * WM * WN;
  constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN, BK = lds_bk<WM, WN, BKO>();
  constexpr int PAD = sizeof(in_t) == 8 ? 8 : 16;
  constexpr int GA = BM * BK / 4, GB = BN * BK / 4;  // 4-element groups per tile
  constexpr int RA = (GA + T - 1) / T, RB = (GB + T - 1) / T;
  __shared__ in_t As[2][BK][BM + PAD];
  __shared__ in_t Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t tn_wg = wg % tm.tiles_n;
  wg /= tm.tiles_n;
  const int64_t tm_wg = wg % tm.tiles_m;
  wg /= tm.tiles_m;
  const int64_t split = (g.batch > 1) ? 0 : wg;
  const int64_t bidx = (g.batch > 1) ? wg : 0;
  const TA *gA = static_cast<const TA *>(g.A) + bidx * g.sA;
  const TB *gB = static_cast<const TB *>(g.B) + bidx * g.sB;
  TC *gC = static_cast<TC *>(g.C) + bidx * g.sC;
  const int64_t M0 = tm_wg * BM, N0 = tn_wg * BN;
  const int64_t kbeg = split * tm.kchunk;
  const int64_t kend = min(g.K, kbeg + tm.kchunk);
  const int r = lane & 15, q = lane >> 4;

  // ---- global -> registers: thread t owns groups t, t + T, ... of 4
  // consecutive elements along the operand's contiguous dimension
  in_t ra[RA][4], rb[RB][4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int t = tid + T * u;
      if (t < GA) {
        int64_t m, k;
        if (AKC) {  // 4 consecutive k of row m
          m = M0 + t / (BK / 4);
          k = k0 + 4 * (t % (BK / 4));
        } else {    // 4 consecutive m of row k
          k = k0 + t / (BM / 4);
          m = M0 + 4 * (t % (BM / 4));
        }
        const TA *p = AKC ? gA + m * g.lda + k : gA + k * g.lda + m;
        const bool full = AKC ? (m < g.M && k + 3 < kend) : (k < kend && m + 3 < g.M);
        if (full && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          load4(p, ra[u]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const bool ok = AKC ? (m < g.M && k + s < kend) : (k < kend && m + s < g.M);
            ra[u][s] = ok ? cvt<in_t>(p[s]) : in_t(0);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int t = tid + T * u;
      if (t < GB) {
        int64_t n, k;
        if (BKC) {
          n = N0 + t / (BK / 4);
          k = k0 + 4 * (t % (BK / 4));
        } else {
          k = k0 + t / (BN / 4);
          n = N0 + 4 * (t % (BN / 4));
        }
        const TB *p = BKC ? gB + n * g.ldb + k : gB + k * g.ldb + n;
        const bool full = BKC ? (n < g.N && k + 3 < kend) : (k < kend && n + 3 < g.N);
        if (full && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          load4(p, rb[u]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const bool ok = BKC ? (n < g.N && k + s < kend) : (k < kend && n + s < g.N);
            rb[u][s] = ok ? cvt<in_t>(p[s]) : in_t(0);
          }
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int t = tid + T * u;
      if (t < GA) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (AKC) As[buf][4 * (t % (BK / 4)) + s][t / (BK / 4)] = ra[u][s];
          else As[buf][t / (BM / 4)][4 * (t % (BM / 4)) + s] = ra[u][s];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int t = tid + T * u;
      if (t < GB) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (BKC) Bs[buf][4 * (t % (BK / 4)) + s][t / (BK / 4)] = rb[u][s];
          else Bs[buf][t / (BN / 4)][4 * (t % (BN / 4)) + s] = rb[u][s];
        }
      }
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  const int am = wm * 16 * TM + r, bn = wn * 16 * TN + r;

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
    in_t a[BK / 4][TM], b[BK / 4][TN];
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
#pragma unroll
      for (int i = 0; i < TM; ++i) a[kk][i] = As[buf][4 * kk + q][am + 16 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[kk][j] = Bs[buf][4 * kk + q][bn + 16 * j];
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MT::mma1(a[kk][i], b[kk][j], acc[i][j]);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // ---- store
  const int64_t m0 = M0 + wm * 16 * TM, n0 = N0 + wn * 16 * TN;
  part_t *part = static_cast<part_t *>(g.partial);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + 16 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int64_t row = m0 + 16 * i + MT::row(q, jj);
        if (row >= g.M) continue;
        const part_t v = acc[i][j][jj];
        if (g.splits > 1) {
          part[(split * g.M + row) * g.N + col] = v;
        } else {
          TC *c = gC + row * g.ldc + col;
          const double out = (g.beta != 0.0)
                                 ? g.alpha * (double)v + g.beta * cvt<double>(*c)
                                 : g.alpha * (double)v;
          *c = (TC)out;
        }
      }
    }
}

// LDS-staged form for the bf16 instruction (v_mfma_f32_16x16x32_bf16: lane
// r + 16 q holds 8 consecutive k, 8 q .. 8 q + 7, of A row r and B column r).
// The tiles are rounded to bf16 (nearest even) as they are staged and kept
// k-contiguous per row of A and per column of B (As[m][k], Bs[n][k], rows
// of 32 + 8 values), so a fragment is one 16-byte LDS read; one MFMA step
// per BK = 32.  A k step's eight products of a lane are summed inside one
// instruction, so the accumulation order differs from the x4 forms.
template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN>
__device__ __forceinline__ void gemm_lds_bf16_body(const GemmX &g, const TileMap &tm,
                                                   int64_t wg) {
  static_assert(MT::CPL == 8, "bf16 instruction");
  typedef typename MT::acc_t acc_t;
  typedef typename MT::part_t part_t;
  constexpr int T = 64 * WM * WN;
  constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN, BK = 32, LDK = BK + 8;
  constexpr int GA = BM * BK / 4, GB = BN * BK / 4;
  constexpr int RA = (GA + T - 1) / T, RB = (GB + T - 1) / T;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN][LDK];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t tn_wg = wg % tm.tiles_n;
  wg /= tm.tiles_n;
  const int64_t tm_wg = wg % tm.tiles_m;
  wg /= tm.tiles_m;
  const int64_t split = (g.batch > 1) ? 0 : wg;
  const int64_t bidx = (g.batch > 1) ? wg : 0;
  const TA *gA = static_cast<const TA *>(g.A) + bidx * g.sA;
  const TB *gB = static_cast<const TB *>(g.B) + bidx * g.sB;
  TC *gC = static_cast<TC *>(g.C) + bidx * g.sC;
  const int64_t M0 = tm_wg * BM, N0 = tn_wg * BN;
  const int64_t kbeg = split * tm.kchunk;
  const int64_t kend = min(g.K, kbeg + tm.kchunk);
  const int r = lane & 15, q = lane >> 4;

  float ra[RA][4], rb[RB][4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int t = tid + T * u;
      if (t < GA) {
        int64_t m, k;
        if (AKC) {
          m = M0 + t / (BK / 4);
          k = k0 + 4 * (t % (BK / 4));
        } else {
          k = k0 + t / (BM / 4);
          m = M0 + 4 * (t % (BM / 4));
        }
        const TA *p = AKC ? gA + m * g.lda + k : gA + k * g.lda + m;
        const bool full = AKC ? (m < g.M && k + 3 < kend) : (k < kend && m + 3 < g.M);
        if (full && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          load4(p, ra[u]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const bool ok = AKC ? (m < g.M && k + s < kend) : (k < kend && m + s < g.M);
            ra[u][s] = ok ? cvt<float>(p[s]) : 0.f;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int t = tid + T * u;
      if (t < GB) {
        int64_t n, k;
        if (BKC) {
          n = N0 + t / (BK / 4);
          k = k0 + 4 * (t % (BK / 4));
        } else {
          k = k0 + t / (BN / 4);
          n = N0 + 4 * (t % (BN / 4));
        }
        const TB *p = BKC ? gB + n * g.ldb + k : gB + k * g.ldb + n;
        const bool full = BKC ? (n < g.N && k + 3 < kend) : (k < kend && n + 3 < g.N);
        if (full && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
          load4(p, rb[u]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const bool ok = BKC ? (n < g.N && k + s < kend) : (k < kend && n + s < g.N);
            rb[u][s] = ok ? cvt<float>(p[s]) : 0.f;
          }
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < RA; ++u) {
      const int t = tid + T * u;
      if (t < GA) {
        if (AKC) {
          const int m = t / (BK / 4), k = 4 * (t % (BK / 4));
#pragma unroll
          for (int s = 0; s < 4; ++s) As[buf][m][k + s] = (__bf16)ra[u][s];
        } else {
          const int k = t / (BM / 4), m = 4 * (t % (BM / 4));
#pragma unroll
          for (int s = 0; s < 4; ++s) As[buf][m + s][k] = (__bf16)ra[u][s];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int t = tid + T * u;
      if (t < GB) {
        if (BKC) {
          const int n = t / (BK / 4), k = 4 * (t % (BK / 4));
#pragma unroll
          for (int s = 0; s < 4; ++s) Bs[buf][n][k + s] = (__bf16)rb[u][s];
        } else {
          const int k = t / (BN / 4), n = 4 * (t % (BN / 4));
#pragma unroll
          for (int s = 0; s < 4; ++s) Bs[buf][n + s][k] = (__bf16)rb[u][s];
        }
      }
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  const int am = wm * 16 * TM + r, bn = wn * 16 * TN + r;

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
    bf8_t a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = *reinterpret_cast<const bf8_t *>(&As[buf][am + 16 * i][8 * q]);
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = *reinterpret_cast<const bf8_t *>(&Bs[buf][bn + 16 * j][8 * q]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  const int64_t m0 = M0 + wm * 16 * TM, n0 = N0 + wn * 16 * TN;
  part_t *part = static_cast<part_t *>(g.partial);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + 16 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int64_t row = m0 + 16 * i + MT::row(q, jj);
        if (row >= g.M) continue;
        const part_t v = acc[i][j][jj];
        if (g.splits > 1) {
          part[(split * g.M + row) * g.N + col] = v;
        } else {
          TC *c = gC + row * g.ldc + col;
          const double out = (g.beta != 0.0)
                                 ? g.alpha * (double)v + g.beta * cvt<double>(*c)
                                 : g.alpha * (double)v;
          *c = (TC)out;
        }
      }
    }
}

// the body for the x4 instructions or the bf16 one
template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN, int BKO>
__device__ __forceinline__ void gemm_any_body(const GemmX &g, const TileMap &tm, int64_t wg) {
  if constexpr (MT::CPL == 4)
    gemm_lds_body<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN, BKO>(g, tm, wg);
  else
    gemm_lds_bf16_body<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN>(g, tm, wg);
}

template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN, int BKO>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(GemmX g, TileMap tm) {
  if (gemm_gated_off(g)) return;
  if (g.sel && *g.sel) {
    g.A = g.A2;
    g.B = g.B2;
  }
  gemm_any_body<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN, BKO>(g, tm, blockIdx.x);
}

// Grouped form: one launch over several independent products (same types,
// layouts and tile shape, any sizes).  Workgroup b belongs to the entry with
// the largest wg_begin <= b.
template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN, int BKO>
__global__ __launch_bounds__(64 * WM * WN) void gemm_group_kernel(const GemmGroupEntry *tab, int count) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].wg_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  const GemmGroupEntry &e = tab[lo];
  TileMap tm;
  tm.tiles_m = e.tiles_m;
  tm.tiles_n = e.tiles_n;
  tm.kchunk = e.kchunk;
  gemm_any_body<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN, BKO>(e.g, tm, b - e.wg_begin);
}

// Sum of the split-K partials into C: 32 output elements per workgroup, the
// eight wavefront-quarters each summing whole groups of eight partials (the
// loads of all of a quarter's groups in flight together), then the group
// sums added in index order.
// Entry blockIdx.y of the table (or the single product g).
constexpr int kRedElems = 32;
constexpr int kRedMaxGroups = 32;  // 256 partials

template <typename TP, typename TC>
__device__ __forceinline__ void splitk_reduce_body(const GemmX &g) {
  __shared__ TP s_gs[kRedMaxGroups][kRedElems];
  const int P = g.splits;
  const int G = (P + kSplitGroup - 1) / kSplitGroup;
  const int64_t total = g.M * g.N;
  const int t = threadIdx.x & (kRedElems - 1), part_of = threadIdx.x / kRedElems;
  const int64_t idx = (int64_t)blockIdx.x * kRedElems + t;
  const bool ok = idx < total;
  const TP *part = static_cast<const TP *>(g.partial);
  // all of a thread's groups are loaded before any is summed, so their loads
  // are in flight together
  constexpr int kQuarters = 256 / kRedElems, kPerQuarter = kRedMaxGroups / kQuarters;
  // (addresses clamped into the buffer and the extra values dropped after
  // the load, so no load sits behind a branch)
  TP v[kPerQuarter][kSplitGroup];
  const int64_t idc = ok ? idx : 0;
#pragma unroll
  for (int h = 0; h < kPerQuarter; ++h) {
    const int grp = part_of + kQuarters * h;
    if (kQuarters * h >= G) break;  // uniform over the workgroup
#pragma unroll
    for (int u = 0; u < kSplitGroup; ++u) {
      const int p = grp * kSplitGroup + u;
      v[h][u] = part[(int64_t)min(p, P - 1) * total + idc];
    }
  }
#pragma unroll
  for (int h = 0; h < kPerQuarter; ++h) {
    if (kQuarters * h >= G) break;
    const int grp = part_of + kQuarters * h;
#pragma unroll
    for (int u = 0; u < kSplitGroup; ++u)
      if (!ok || grp * kSplitGroup + u >= P) v[h][u] = TP(0);
  }
#pragma unroll
  for (int h = 0; h < kPerQuarter; ++h) {
    const int grp = part_of + kQuarters * h;
    if (grp >= G) break;
    TP gs = TP(0);
#pragma unroll
    for (int u = 0; u < kSplitGroup; ++u) gs += v[h][u];
    s_gs[grp][t] = gs;
  }
  __syncthreads();
  if (part_of != 0 || !ok) return;
  TP acc = s_gs[0][t];
  if (G > 1) {
    acc = TP(0);
    for (int grp = 0; grp < G; ++grp) acc += s_gs[grp][t];
  }
  const int64_t row = idx / g.N, col = idx - row * g.N;
  TC *c = static_cast<TC *>(g.C) + row * g.ldc + col;
  const double out = (g.beta != 0.0) ? g.alpha * (double)acc + g.beta * cvt<double>(*c)
                                     : g.alpha * (double)acc;
  *c = (TC)out;
}

template <typename TP, typename TC>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmX g) {
  if (gemm_gated_off(g)) return;
  splitk_reduce_body<TP, TC>(g);
}

template <typename TP, typename TC>
__global__ __launch_bounds__(256) void splitk_group_reduce_kernel(const GemmGroupEntry *tab) {
  const GemmX &g = tab[blockIdx.y].g;
  if (g.splits <= 1 || (int64_t)blockIdx.x * kRedElems >= g.M * g.N) return;
  splitk_reduce_body<TP, TC>(g);
}

struct Variant {
  int tm, tn, wm, wn;
};
// Output tile per workgroup, every arithmetic: 32x64, 64x32 (eight
// wavefronts each, K steps of 16), 64x64, 128x128 (four wavefronts each, K
// steps of 32); variants 4 and 5 are the eight-wavefront tiles with K steps
// of 32, which the single path takes for grids of at most kDeepGrid
// workgroups (half the steps, and occupancy matters less in a grid that
// does not fill the CUs twice)
constexpr Variant kVarLds[] = {{1, 1, 2, 4}, {1, 1, 4, 2}, {2, 2, 2, 2},
                               {4, 4, 2, 2}, {1, 1, 2, 4}, {1, 1, 4, 2}};
constexpr int64_t kDeepGrid = 320;

const Variant &variant_of(DType math, int v) {
  (void)math;  // one table for every arithmetic
  return kVarLds[v];
}

void tile_of(DType math, int v, int64_t *bm, int64_t *bn) {
  const Variant &x = variant_of(math, v);
  *bm = 16 * x.tm * x.wm;
  *bn = 16 * x.tn * x.wn;
}

int pick_variant(int64_t M, int64_t N, DType math) {
  // least padded work; ties go to the smaller tile (more workgroups)
  int best = 0;
  double best_cost = 1e300;
  for (int v = 0; v < 4; ++v) {
    int64_t bm, bn;
    tile_of(math, v, &bm, &bn);
    const double cost = double((M + bm - 1) / bm * bm) * double((N + bn - 1) / bn * bn) *
                        (1.0 + 1e-3 * (double)(bm * bn));
    if (cost < best_cost) {
      best_cost = cost;
      best = v;
    }
  }
  return best;
}

template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC, int TM, int TN,
          int WM, int WN, int BKO = 0>
void launch_one(const GemmX &g, const TileMap &tm, int64_t grid, hipStream_t s,
                const GemmGroupEntry *tab, int count) {
  const dim3 gr((unsigned)grid), bl(64 * WM * WN);
  if (tab)
    hipLaunchKernelGGL((gemm_group_kernel<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN, BKO>), gr, bl,
                       0, s, tab, count);
  else
    hipLaunchKernelGGL((gemm_kernel<MT, TA, TB, TC, AKC, BKC, TM, TN, WM, WN, BKO>), gr, bl, 0, s,
                       g, tm);
}

template <class MT, typename TA, typename TB, typename TC, bool AKC, bool BKC>
void launch_layout(int v, const GemmX &g, const TileMap &tm, int64_t grid, hipStream_t s,
                   const GemmGroupEntry *tab, int count) {
  switch (v) {
    case 0:
      launch_one<MT, TA, TB, TC, AKC, BKC, 1, 1, 2, 4>(g, tm, grid, s, tab, count);
      break;
    case 1:
      launch_one<MT, TA, TB, TC, AKC, BKC, 1, 1, 4, 2>(g, tm, grid, s, tab, count);
      break;
    case 2:
      launch_one<MT, TA, TB, TC, AKC, BKC, 2, 2, 2, 2>(g, tm, grid, s, tab, count);
      break;
    case 4:
      launch_one<MT, TA, TB, TC, AKC, BKC, 1, 1, 2, 4, 32>(g, tm, grid, s, tab, count);
      break;
    case 5:
      launch_one<MT, TA, TB, TC, AKC, BKC, 1, 1, 4, 2, 32>(g, tm, grid, s, tab, count);
      break;
    default:
      launch_one<MT, TA, TB, TC, AKC, BKC, 4, 4, 2, 2>(g, tm, grid, s, tab, count);
      break;
  }
}

template <class MT, typename TA, typename TB, typename TC>
void launch_types(int v, const GemmX &g, const TileMap &tm, int64_t grid, hipStream_t s,
                  const GemmGroupEntry *tab, int count) {
  if (g.a_kc) {
    if (g.b_kc) launch_layout<MT, TA, TB, TC, true, true>(v, g, tm, grid, s, tab, count);
    else launch_layout<MT, TA, TB, TC, true, false>(v, g, tm, grid, s, tab, count);
  } else {
    if (g.b_kc) launch_layout<MT, TA, TB, TC, false, true>(v, g, tm, grid, s, tab, count);
    else launch_layout<MT, TA, TB, TC, false, false>(v, g, tm, grid, s, tab, count);
  }
}

constexpr int tkey(DType m, DType a, DType b, DType c) {
  return ((int)m << 6) | ((int)a << 4) | ((int)b << 2) | (int)c;
}

// the type combinations the rounding uses
bool dispatch(int v, const GemmX &g, const TileMap &tm, int64_t grid, hipStream_t s,
              const GemmGroupEntry *tab = nullptr, int count = 0) {
  using D = DType;
  switch (tkey(g.math, g.ta, g.tb, g.tc)) {
    case tkey(D::F64, D::F64, D::F64, D::F64):
      launch_types<MathF64, double, double, double>(v, g, tm, grid, s, tab, count);
      return true;
    case tkey(D::F64, D::F32, D::F32, D::F64):
      launch_types<MathF64, float, float, double>(v, g, tm, grid, s, tab, count);
      return true;
    case tkey(D::F64, D::F64, D::F32, D::F32):  // FP64 factor times FP32 storage
      launch_types<MathF64, double, float, float>(v, g, tm, grid, s, tab, count);
      return true;
    case tkey(D::F32, D::F32, D::F32, D::F32):
      launch_types<MathF32, float, float, float>(v, g, tm, grid, s, tab, count);
      return true;
    case tkey(D::BF16, D::F32, D::F32, D::F32):
      launch_types<MathBF16, float, float, float>(v, g, tm, grid, s, tab, count);
      return true;
    case tkey(D::BF16, D::F32, D::BF16, D::F32):
      launch_types<MathBF16, float, __bf16, float>(v, g, tm, grid, s, tab, count);
      return true;
    default:
      return false;
  }
}

}  // namespace

int gemm_chunk(DType math) { return math == DType::BF16 ? 32 : 16; }



int gemm_pick_splits(int64_t M, int64_t N, int64_t K, DType math) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  const int v = pick_variant(M, N, math);
  int64_t bm, bn;
  tile_of(math, v, &bm, &bn);
  const int64_t wgs = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  const int64_t want = 512;  // workgroups: 2 per CU
  if (wgs >= want / 2) return 1;
  int64_t sp = (want + wgs - 1) / wgs;
  const int64_t max_by_k = std::max<int64_t>(1, K / 128);  // >= 4 K-chunks each
  sp = std::min(sp, max_by_k);
  sp = std::min<int64_t>(sp, 256);
  return (int)std::max<int64_t>(1, sp);
}

size_t gemm_acc_bytes(DType math) { return math == DType::F64 ? 8 : 4; }

static int64_t split_kchunk(const GemmX &g) {
  const int splits = std::max(1, g.splits);
  const int chunk = gemm_chunk(g.math);
  int64_t kchunk = (g.K + splits - 1) / splits;
  return (kchunk + chunk - 1) / chunk * chunk;
}

int gemm_used_splits(const GemmX &g) {
  if (g.K <= 0 || g.batch > 1) return 1;
  const int64_t kchunk = split_kchunk(g);
  return (int)((g.K + kchunk - 1) / kchunk);
}

int gemmx_run(const GemmX &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return TT_OK;
  if (g.K <= 0) return fail(TT_EINVAL, "gemm with K <= 0");
  if (g.batch > 1 && g.splits > 1) return fail(TT_EINVAL, "batched split-K gemm");
  if (g.batch < 1) return TT_OK;
  const int v = pick_variant(g.M, g.N, g.math);
  int64_t bm, bn;
  tile_of(g.math, v, &bm, &bn);
  TileMap tm;
  tm.tiles_m = (g.M + bm - 1) / bm;
  tm.tiles_n = (g.N + bn - 1) / bn;
  const int64_t kchunk = split_kchunk(g);
  const int64_t used_splits = (g.K + kchunk - 1) / kchunk;
  GemmX gg = g;
  gg.splits = (int)used_splits;
  tm.kchunk = kchunk;
  if (gg.splits > 1 && gg.partial == nullptr) return fail(TT_EINVAL, "split-K without buffer");
  if (gg.splits > kRedMaxGroups * kSplitGroup) return fail(TT_EINVAL, "internal: too many K splits");
  const int64_t grid = tm.tiles_m * tm.tiles_n * (g.batch > 1 ? g.batch : used_splits);
  const int vv = (v <= 1 && grid <= kDeepGrid && g.math != DType::BF16) ? v + 4 : v;
  if (!dispatch(vv, gg, tm, grid, s)) return fail(TT_EINVAL, "internal: gemm type combination");
  TTR_HIP(hipGetLastError());
  if (gg.splits > 1) TTR_TRY(gemm_reduce_splits(gg, s));
  return TT_OK;
}

int gemm_reduce_splits(const GemmX &g, hipStream_t s) {
  if (g.splits <= 1 || g.M <= 0 || g.N <= 0) return TT_OK;
  if (!g.partial) return fail(TT_EINVAL, "internal: split sum without partials");
  if (g.splits > kRedMaxGroups * kSplitGroup) return fail(TT_EINVAL, "internal: too many K splits");
  const int64_t total = g.M * g.N;
  const dim3 gr((unsigned)((total + kRedElems - 1) / kRedElems)), bl(256);
  if (g.math == DType::F64) {
    if (g.tc == DType::F64)
      hipLaunchKernelGGL((splitk_reduce_kernel<double, double>), gr, bl, 0, s, g);
    else
      hipLaunchKernelGGL((splitk_reduce_kernel<double, float>), gr, bl, 0, s, g);
  } else {
    if (g.tc == DType::F64)
      hipLaunchKernelGGL((splitk_reduce_kernel<float, double>), gr, bl, 0, s, g);
    else
      hipLaunchKernelGGL((splitk_reduce_kernel<float, float>), gr, bl, 0, s, g);
  }
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int gemm_variant_count() { return 4; }

void gemm_variant_tile(DType math, int v, int64_t *bm, int64_t *bn) { tile_of(math, v, bm, bn); }

int gemm_group_splits(const GemmX &g) {
  // bound the K range of one workgroup (~512) so that long contractions of
  // small outputs (Gram matrices, projections) spread over many workgroups
  if (g.K <= 1024) return 1;
  return (int)std::min<int64_t>(64, (g.K + 511) / 512);
}

int gemm_group_fill(const GemmX &g, int v, int64_t wg_begin, GemmGroupEntry *e) {
  if (g.M <= 0 || g.N <= 0) return fail(TT_EINVAL, "grouped gemm with an empty product");
  if (g.K <= 0) return fail(TT_EINVAL, "grouped gemm with K <= 0");
  if (g.batch > 1) return fail(TT_EINVAL, "grouped gemm entries are single products");
  int64_t bm, bn;
  gemm_variant_tile(g.math, v, &bm, &bn);
  e->g = g;
  e->tiles_m = (g.M + bm - 1) / bm;
  e->tiles_n = (g.N + bn - 1) / bn;
  const int chunk = gemm_chunk(g.math);
  const int sp = (g.partial && g.splits > 1) ? g.splits : 1;
  int64_t kc = (g.K + sp - 1) / sp;
  kc = (kc + chunk - 1) / chunk * chunk;
  e->kchunk = kc;
  e->g.splits = (int)((g.K + kc - 1) / kc);
  if (e->g.splits <= 1) {
    e->g.splits = 1;
    e->g.partial = nullptr;
  }
  if (e->g.splits > kRedMaxGroups * kSplitGroup) return fail(TT_EINVAL, "internal: too many K splits");
  e->wg_begin = wg_begin;
  return TT_OK;
}

int64_t gemm_group_wgs(const GemmGroupEntry &e) { return e.tiles_m * e.tiles_n * e.g.splits; }

int gemm_group_reduce(const GemmX &rep, const GemmGroupEntry *d_tab, int count, int64_t max_mn,
                      hipStream_t s) {
  if (count <= 0 || max_mn <= 0) return TT_OK;
  const dim3 gr((unsigned)((max_mn + kRedElems - 1) / kRedElems), (unsigned)count), bl(256);
  if (rep.math == DType::F64) {
    if (rep.tc == DType::F64)
      hipLaunchKernelGGL((splitk_group_reduce_kernel<double, double>), gr, bl, 0, s, d_tab);
    else
      hipLaunchKernelGGL((splitk_group_reduce_kernel<double, float>), gr, bl, 0, s, d_tab);
  } else {
    if (rep.tc == DType::F64)
      hipLaunchKernelGGL((splitk_group_reduce_kernel<float, double>), gr, bl, 0, s, d_tab);
    else
      hipLaunchKernelGGL((splitk_group_reduce_kernel<float, float>), gr, bl, 0, s, d_tab);
  }
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

int gemm_group_run(const GemmX &rep, int v, const GemmGroupEntry *d_tab, int count,
                   int64_t total_wgs, hipStream_t s) {
  if (count <= 0 || total_wgs <= 0) return TT_OK;
  TileMap tm{};
  if (!dispatch(v, rep, tm, total_wgs, s, d_tab, count))
    return fail(TT_EINVAL, "internal: gemm type combination");
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

}  // namespace ttr
