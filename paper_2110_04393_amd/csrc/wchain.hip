// One level of the partial contractions of Algorithm 3 in a single kernel,
// for every summand of a sum (Algorithm 7) at once.
//
// For a TT Y (core n: R0 x I x R1), the sketch core Sk_n (L0 x I x L1) and
// W_n (R1 x L1) it computes
//   W_{n-1}(a, b) = sum_i sum_c Z(a, i, c) Sk_n(b, i, c),
//   Z(a, i, c)    = sum_k Y_n(a, i, k) W_n(k, c),
// i.e. W_{n-1} = H(V(Y_n) W_n) H(Sk_n)^T (the two products of one step of
// the recursion that defines W_n), without writing Z = V(Y_n) W_n to memory.
//
// Work decomposition.  A unit is (16 consecutive a, one i): its Z block is
// 16 x L1.  A workgroup owns one 16-row a-block of one summand and a range of
// i; it holds that summand's W_n^T in LDS (all of it: L1 rows, R1 columns).
// Its wavefronts form NCB c-block columns (4 for L1 <= 64, else 8; blocks
// past L1 are zero) x ULN unit lanes; a lane takes the units i, i + ULN, ...
// of the range.  Per unit, the wavefront of c-block cb
//   1. forms Z^T(c-block, a-block) = W^T(c-block, :) Y_i^T (:, a-block) with
//      the x4 MFMA instruction of the arithmetic (W^T fragments from LDS, Y
//      staged through LDS: in each batch of NCB 16-wide k-chunks every
//      wavefront of the lane loads one chunk with raw buffer loads and all of
//      them read it after one barrier; the next batch is in flight meanwhile),
//   2. multiplies its accumulator, still in registers, by Sk_n(:, i, c-block)^T
//      into the running W_{n-1}(a-block, :) accumulator (the Sk fragments of a
//      unit are loaded while the previous unit runs).
// Step 2 needs lane (r, q) of the accumulator to hold Z(a0 + r, c) for four
// consecutive c: the accumulator of the f32 instruction holds rows 4 q + j
// already; for the f64 instruction (rows q + 4 j) the W^T rows are staged in
// the permuted order m -> 4 (m % 4) + m / 4, which gives the same property.
// At the end the wavefronts' accumulators are summed in LDS in a fixed order
// and written as one i-range split of the result (added in split order by
// wfuse_sum_kernel) or directly when there is one range.  The BF16 form
// (wfuse_bf16_kernel) follows the same plan with the bf16 instruction.
#include <algorithm>
#include <type_traits>

#include "tt_internal.h"
#include "wave.h"

namespace ttr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

struct FuseF64 {
  typedef double T;
  typedef d4_t acc_t;
  __device__ static acc_t mma(T a, T b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator row of register j in lane quad q
  __device__ static int row(int q, int j) { return q + 4 * j; }
  // c offset (within a 16-block) staged in W^T row m
  __host__ __device__ static int perm(int m) { return 4 * (m & 3) + (m >> 2); }
  __device__ static void store4(T *p, const T (&v)[4]) {
    *reinterpret_cast<d2_t *>(p) = d2_t{v[0], v[1]};
    *reinterpret_cast<d2_t *>(p + 2) = d2_t{v[2], v[3]};
  }
  __device__ static void load4(const T *p, T (&o)[4]) {
    const d2_t x = *reinterpret_cast<const d2_t *>(p);
    const d2_t y = *reinterpret_cast<const d2_t *>(p + 2);
    o[0] = x[0];
    o[1] = x[1];
    o[2] = y[0];
    o[3] = y[1];
  }
};
struct FuseF32 {
  typedef float T;
  typedef f4_t acc_t;
  __device__ static acc_t mma(T a, T b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int q, int j) { return 4 * q + j; }
  __host__ __device__ static int perm(int m) { return m; }
  __device__ static void store4(T *p, const T (&v)[4]) {
    *reinterpret_cast<f4_t *>(p) = f4_t{v[0], v[1], v[2], v[3]};
  }
  __device__ static void load4(const T *p, T (&o)[4]) {
    const f4_t x = *reinterpret_cast<const f4_t *>(p);
    o[0] = x[0];
    o[1] = x[1];
    o[2] = x[2];
    o[3] = x[3];
  }
};

// One summand of a level: its core Y^(j)_n (R0 x I x R1), its rows of the
// stacked W_n (R1 x L1, ld L1), where its W_(n-1) block or its splits go,
// and the first of its tiles (a-block x i-range) in the launch.
constexpr int kFuseMaxGroup = 24;
struct WFuseEntry {
  const void *Y, *W;
  void *out;  // W_(n-1) rows (ld L0) with one i-range, else its splits [groups][R0][L0]
  int32_t R0, R1, nch, ldk, nablk, tile0;
};
struct WFuseArgs {
  const void *Sk;
  int64_t I, L1, L0, ipg;
  int ncb, nbb, uln, direct, count;
  WFuseEntry e[kFuseMaxGroup];
};

extern __shared__ __attribute__((aligned(16))) unsigned char wf_lds[];

// Operands are read with raw buffer loads: a lane whose fragment lies outside
// the operand passes an offset beyond the buffer's size and reads zeros, so
// every lane issues the same loads (no branches, and the waits on the
// in-order load counter stay exact).
constexpr uint32_t kOutside = 0x80000000u;  // beyond every buffer (< 2 GiB)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  // dword 3: 32-bit data format, as for untyped loads on gfx9-class parts
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&o)[4]) {
  const u4_t x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  const u4_t y = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
  const d2_t a = __builtin_bit_cast(d2_t, x), b = __builtin_bit_cast(d2_t, y);
  o[0] = a[0];
  o[1] = a[1];
  o[2] = b[0];
  o[3] = b[1];
}
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[4]) {
  const f4_t a = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  o[0] = a[0];
  o[1] = a[1];
  o[2] = a[2];
  o[3] = a[3];
}
__device__ __forceinline__ double bload1(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bload1(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <class F, int NCB, int NBB, int ULN, bool VS>
__global__ __launch_bounds__(64 * NCB * ULN) void wfuse_kernel(const WFuseArgs p) {
  typedef typename F::T T;
  typedef typename F::acc_t acc_t;
  // staged Y rows: 16 values + one 16-byte step, which spreads a fragment
  // read over the LDS banks and keeps rows 16-byte aligned
  constexpr int YR = 16 + 16 / (int)sizeof(T);
  constexpr int POS = 16 * YR;  // values of one staged position (16 rows)
  T *Wt = reinterpret_cast<T *>(wf_lds);
  const T *Sk = static_cast<const T *>(p.Sk);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, q = lane >> 4;
  const int cb = wave % NCB, ul = wave / NCB;
  // Workgroup b runs on XCD b % 8 (round-robin dispatch); each XCD takes a
  // contiguous run of the (i-range, a-block) tiles, so the a-blocks of one
  // i-range, which share Sk_n(:, i-range, :), mostly share one L2.
  int tile;
  {
    const int nwg = gridDim.x, b = blockIdx.x;
    const int per = nwg / 8, extra = nwg % 8, x = b % 8;
    tile = x * per + min(x, extra) + b / 8;
  }
  // the summand of this tile (tiles are numbered summand by summand)
  int j = 0;
  while (j + 1 < p.count && tile >= p.e[j + 1].tile0) ++j;
  const WFuseEntry &ent = p.e[j];
  const T *Y = static_cast<const T *>(ent.Y);
  const T *W = static_cast<const T *>(ent.W);
  const int64_t R0 = ent.R0, R1_ = ent.R1;
  const int ldk = ent.ldk, nablk = ent.nablk;
  tile -= ent.tile0;
  const int64_t ab = tile % nablk, grp = tile / nablk;
  const int64_t a0 = 16 * ab;
  const int64_t ib = grp * p.ipg, ie = min(p.I, ib + p.ipg);
  const int rows = 16 * NCB, kp = 16 * ent.nch;
  const int nch = ent.nch;
  // staged Y: per unit lane two buffers of NCB positions, after W^T
  T *Ys = Wt + rows * ldk + ul * 2 * NCB * POS;

  // units of this lane: i = ib + ul, ib + ul + ULN, ... (< ie)
  const int64_t left = ie - ib - ul;
  const int nu = left > 0 ? (int)((left + ULN - 1) / ULN) : 0;
  // the chunks of a unit are padded to nchp, a multiple of 8 (so of NCB):
  // a batch is NCB consecutive positions of one unit, position NCB g + w of
  // batch g is loaded by wavefront w of the lane
  const int nchp = (nch + 7) / 8 * 8;
  const int bpu = nchp / NCB;  // batches per unit
  const int64_t arow = a0 + r;
  const bool arow_ok = arow < R0;
  constexpr uint32_t es = sizeof(T);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y, (uint32_t)(R0 * p.I * R1_ * es));
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(Sk, (uint32_t)(p.L0 * p.I * p.L1 * es));

  // Y fragment of this wavefront's position in batch g: lane (r, q) holds
  // Y(a0 + r, i, 16 c + 4 q + t); R1 is a multiple of 4, so the four values
  // are all inside the row or all outside (chunks c >= nch, units u >= nu
  // and rows beyond R0 read zeros).  Offsets fit in 32 bits.
  const uint32_t R1 = (uint32_t)R1_, L1 = (uint32_t)p.L1, I = (uint32_t)p.I;
  const uint32_t y_lane = ((uint32_t)arow * I * R1 + 4 * q) * es;
  auto loady = [&](int g, T(&v)[4]) __attribute__((always_inline)) {
    const int u = g / bpu, c = (g - u * bpu) * NCB + cb;
    const uint32_t i = (uint32_t)(ib + ul) + (uint32_t)u * ULN;
    const bool ok = arow_ok && u < nu && c < nch && 16 * c + 4 * q < (int)R1;
    bload4(ry, ok ? y_lane + (i * R1 + 16 * c) * es : kOutside, v);
  };
  // the wavefront's staged position of buffer b: row r, values 4 q .. 4 q + 3
  auto stagey = [&](int b, const T(&v)[4]) __attribute__((always_inline)) {
    F::store4(Ys + (b * NCB + cb) * POS + r * YR + 4 * q, v);
  };
  // Sk fragments of unit u: lane (r, q) holds Sk(16 bb + r, i, cc + j)
  const int cc = 16 * cb + 4 * q;  // first c of this lane's P2 k-slots
  const uint32_t s_lane = ((uint32_t)r * I * L1 + cc) * es;
  auto loadsk = [&](int u, T(&v)[NBB][4]) __attribute__((always_inline)) {
    const uint32_t i = (uint32_t)(ib + ul) + (uint32_t)u * ULN;
#pragma unroll
    for (int bb = 0; bb < NBB; ++bb) {
      const bool bok = u < nu && 16 * bb + r < p.L0;
      const uint32_t off = s_lane + (16 * bb * I + i) * L1 * es;
      if constexpr (VS) {
        // L1 is a multiple of 4: the four values are inside the row or not
        bload4(rs, bok && cc < (int)L1 ? off : kOutside, v[bb]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          v[bb][j] = bload1(rs, bok && cc + j < (int)L1 ? off + j * es : kOutside, T(0));
      }
    }
  };

  // batches 0 and 1 and the first unit's Sk fragments go out first
  T yr[2][4];
  T sk[NBB][4];
  loady(0, yr[0]);
  loady(1, yr[1]);
  loadsk(0, sk);

  // W^T into LDS: row m holds column 16 (m / 16) + perm(m % 16) of W_n,
  // zero beyond R1 and L1 (so padded k and c contribute nothing); sixteen
  // loads per thread in flight before their LDS stores
  {
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(W, (uint32_t)(R1_ * p.L1 * es));
    constexpr int kBatch = 16;
    const int n = rows * kp, step = blockDim.x;
    for (int e0 = tid; e0 < n; e0 += kBatch * step) {
      T v[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * step;
        const int k = e / rows, m = e - k * rows;
        const int c = 16 * (m >> 4) + F::perm(m & 15);
        const bool ok = e < n && k < R1_ && c < p.L1;
        v[b] = bload1(rw, ok ? (uint32_t)(((int64_t)k * p.L1 + c) * es) : kOutside, T(0));
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * step;
        const int k = e / rows, m = e - k * rows;
        if (e < n) Wt[m * ldk + k] = v[b];
      }
    }
  }
  stagey(0, yr[0]);
  __syncthreads();

  acc_t acc1[2], acc2[NBB];
  acc1[0] = acc1[1] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int bb = 0; bb < NBB; ++bb) acc2[bb] = acc_t{0, 0, 0, 0};
  const T *wrow = Wt + (16 * cb + r) * ldk + 4 * q;
  const T *yfrag = Ys + r * YR + 4 * q;
  // with eight c-blocks (L1 > 64), c-blocks past L1 and b-blocks past L0
  // (padding of the tile shape) hold zeros: their wavefronts only load and
  // stage, and no product runs on them (the four-block form keeps its
  // branch-free products)
  const bool cb_live = NCB == 4 || 16 * cb < (int)p.L1;

  // Batch g (buffer g % 2): issue the loads of batch g + 2 into the
  // registers of batch g (already staged), run the NCB positions of batch g
  // from LDS, stage batch g + 1 into the other buffer, barrier.  Each unit
  // ends with its Sk product.  All wavefronts run the same number of
  // batches (units past the lane's last read zeros), so the barriers match.
  const int nbw = (int)((p.ipg + ULN - 1) / ULN) * bpu;  // batches of every lane
  int g = 0;
  for (int u = 0; u * bpu < nbw; ++u) {
    for (int bi = 0; bi < bpu; ++bi, ++g) {
      const int b = g & 1;
      if (b == 0) loady(g + 2, yr[0]); else loady(g + 2, yr[1]);
      static_for<0, NCB>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const int c = bi * NCB + s;
        if (c < nch && cb_live) {
          T w[4], y[4];
          F::load4(wrow + 16 * c, w);
          F::load4(yfrag + (b * NCB + s) * POS, y);
#pragma unroll
          for (int t = 0; t < 4; ++t) acc1[t & 1] = F::mma(w[t], y[t], acc1[t & 1]);
        }
      });
      if (b == 0) stagey(1, yr[1]); else stagey(0, yr[0]);
      __syncthreads();
    }
    // unit complete: Z(a0 + r, i, cc + j) = register j of the sum; b-blocks
    // beyond L0 multiply zeros
    const acc_t z = acc1[0] + acc1[1];
    acc1[0] = acc1[1] = acc_t{0, 0, 0, 0};
    if constexpr (NCB == 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int bb = 0; bb < NBB; ++bb) acc2[bb] = F::mma(z[j], sk[bb][j], acc2[bb]);
    } else if (cb_live) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int bb = 0; bb < NBB; ++bb)
          if (bb < p.nbb) acc2[bb] = F::mma(z[j], sk[bb][j], acc2[bb]);
    }
    loadsk(u + 1, sk);
  }

  // sum of the wavefronts' W_{n-1}(a-block, :) in wavefront order
  __syncthreads();
  T *red = reinterpret_cast<T *>(wf_lds);
  const int ncol = 16 * p.nbb;
#pragma unroll
  for (int bb = 0; bb < NBB; ++bb)
    if (bb < p.nbb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) red[(wave * 16 + F::row(q, j)) * ncol + 16 * bb + r] = acc2[bb][j];
    }
  __syncthreads();
  const int waves = blockDim.x >> 6;
  T *out = static_cast<T *>(ent.out);
  for (int e = tid; e < 16 * p.L0; e += blockDim.x) {
    const int rr = e / (int)p.L0, col = e - rr * (int)p.L0;
    const int64_t a = a0 + rr;
    if (a >= R0) continue;
    T acc = T(0);
    for (int w = 0; w < waves; ++w) acc += red[(w * 16 + rr) * ncol + col];
    if (p.direct)
      out[a * p.L0 + col] = acc;
    else
      out[(grp * R0 + a) * p.L0 + col] = acc;
  }
}

// BF16 form of the same kernel (mixed precision: cores and W in FP32
// storage, the sketch in BF16 or FP32 storage, products on the BF16
// instruction with FP32 accumulation).  Y and W_n are rounded to BF16 (nearest
// even) as they are staged in LDS; a position is 32 values of k and one
// v_mfma_f32_16x16x32_bf16, whose lane (r, q) holds 8 consecutive k,
// 8 q .. 8 q + 7, of its row or column.  The FP32 accumulator already holds
// rows 4 q + j, so W^T rows keep their order; the second product rounds
// Z(a0 + r, cc + j) to BF16 and fills the lane's other four k-slots with
// zeros (16 real k per instruction).
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned short us4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bload1f(__amdgpu_buffer_rsrc_t r, uint32_t off, __bf16) {
  const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
  return (float)__builtin_bit_cast(__bf16, v);
}
__device__ __forceinline__ float bload1f(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// four consecutive sketch values (16 bytes of FP32 or 8 bytes of BF16)
__device__ __forceinline__ void bload4f(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[4],
                                        float) {
  const f4_t a = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  o[0] = a[0];
  o[1] = a[1];
  o[2] = a[2];
  o[3] = a[3];
}
__device__ __forceinline__ void bload4f(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[4],
                                        __bf16) {
  const u2_t x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  const us4_t h = __builtin_bit_cast(us4_t, x);
#pragma unroll
  for (int t = 0; t < 4; ++t) o[t] = (float)__builtin_bit_cast(__bf16, (unsigned short)h[t]);
}
__device__ __forceinline__ bf8_t bf16_lo4(const float (&v)[4]) {
  return bf8_t{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3],
               (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
}

template <int NCB, int NBB, int ULN, bool VS, typename TS>
__global__ __launch_bounds__(64 * NCB * ULN) void wfuse_bf16_kernel(const WFuseArgs p) {
  constexpr int YR = 40;        // staged Y row: 32 values + 16 bytes
  constexpr int POS = 16 * YR;  // values of one staged position (16 rows)
  __bf16 *Wt = reinterpret_cast<__bf16 *>(wf_lds);
  const TS *Sk = static_cast<const TS *>(p.Sk);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, q = lane >> 4;
  const int cb = wave % NCB, ul = wave / NCB;
  int tile;
  {
    const int nwg = gridDim.x, b = blockIdx.x;
    const int per = nwg / 8, extra = nwg % 8, x = b % 8;
    tile = x * per + min(x, extra) + b / 8;
  }
  int j = 0;
  while (j + 1 < p.count && tile >= p.e[j + 1].tile0) ++j;
  const WFuseEntry &ent = p.e[j];
  const float *Y = static_cast<const float *>(ent.Y);
  const float *W = static_cast<const float *>(ent.W);
  const int64_t R0 = ent.R0, R1_ = ent.R1;
  const int ldk = ent.ldk, nablk = ent.nablk;
  tile -= ent.tile0;
  const int64_t ab = tile % nablk, grp = tile / nablk;
  const int64_t a0 = 16 * ab;
  const int64_t ib = grp * p.ipg, ie = min(p.I, ib + p.ipg);
  const int rows = 16 * NCB, nch = ent.nch, kp = 32 * nch;
  __bf16 *Ys = Wt + rows * ldk + ul * 2 * NCB * POS;

  const int64_t left = ie - ib - ul;
  const int nu = left > 0 ? (int)((left + ULN - 1) / ULN) : 0;
  const int nchp = (nch + 7) / 8 * 8;
  const int bpu = nchp / NCB;
  const int64_t arow = a0 + r;
  const bool arow_ok = arow < R0;
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(Y, (uint32_t)(R0 * p.I * R1_ * 4));
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(Sk, (uint32_t)(p.L0 * p.I * p.L1 * sizeof(TS)));
  const uint32_t R1 = (uint32_t)R1_, L1 = (uint32_t)p.L1, I = (uint32_t)p.I;
  const uint32_t y_lane = ((uint32_t)arow * I * R1 + 8 * q) * 4;
  // Y of this wavefront's position in batch g: Y(a0 + r, i, 32 c + 8 q + t),
  // as two 4-vectors (R1 is a multiple of 4)
  auto loady = [&](int g, float(&v)[8]) __attribute__((always_inline)) {
    const int u = g / bpu, c = (g - u * bpu) * NCB + cb;
    const uint32_t i = (uint32_t)(ib + ul) + (uint32_t)u * ULN;
    const int k = 32 * c + 8 * q;
    const bool ok = arow_ok && u < nu && c < nch;
    const uint32_t off = y_lane + (i * R1 + 32 * c) * 4;
    const f4_t lo = __builtin_bit_cast(
        f4_t, __builtin_amdgcn_raw_buffer_load_b128(ry, ok && k < (int)R1 ? off : kOutside, 0, 0));
    const f4_t hi = __builtin_bit_cast(
        f4_t,
        __builtin_amdgcn_raw_buffer_load_b128(ry, ok && k + 4 < (int)R1 ? off + 16 : kOutside, 0, 0));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v[t] = lo[t];
      v[t + 4] = hi[t];
    }
  };
  auto stagey = [&](int b, const float(&v)[8]) __attribute__((always_inline)) {
    *reinterpret_cast<bf8_t *>(Ys + (b * NCB + cb) * POS + r * YR + 8 * q) =
        bf8_t{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3],
              (__bf16)v[4], (__bf16)v[5], (__bf16)v[6], (__bf16)v[7]};
  };
  const int cc = 16 * cb + 4 * q;
  const uint32_t s_lane = ((uint32_t)r * I * L1 + cc) * (uint32_t)sizeof(TS);
  auto loadsk = [&](int u, float(&v)[NBB][4]) __attribute__((always_inline)) {
    const uint32_t i = (uint32_t)(ib + ul) + (uint32_t)u * ULN;
#pragma unroll
    for (int bb = 0; bb < NBB; ++bb) {
      const bool bok = u < nu && 16 * bb + r < p.L0;
      const uint32_t off = s_lane + (16 * bb * I + i) * L1 * (uint32_t)sizeof(TS);
      if constexpr (VS) {
        bload4f(rs, bok && cc < (int)L1 ? off : kOutside, v[bb], TS(0));
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          v[bb][t] = bload1f(rs, bok && cc + t < (int)L1 ? off + t * (uint32_t)sizeof(TS) : kOutside,
                             TS(0));
      }
    }
  };

  float yr[2][8];
  float sk[NBB][4];
  loady(0, yr[0]);
  loady(1, yr[1]);
  loadsk(0, sk);
  // W^T into LDS (row m = column m of W_n), rounded to BF16, zero beyond R1
  // and L1
  {
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(W, (uint32_t)(R1_ * p.L1 * 4));
    constexpr int kBatch = 16;
    const int n = rows * kp, step = blockDim.x;
    for (int e0 = tid; e0 < n; e0 += kBatch * step) {
      float v[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * step;
        const int k = e / rows, m = e - k * rows;
        const bool ok = e < n && k < R1_ && m < p.L1;
        v[b] = bload1(rw, ok ? (uint32_t)(((int64_t)k * p.L1 + m) * 4) : kOutside, 0.f);
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * step;
        const int k = e / rows, m = e - k * rows;
        if (e < n) Wt[m * ldk + k] = (__bf16)v[b];
      }
    }
  }
  stagey(0, yr[0]);
  __syncthreads();

  f4_t acc1[2], acc2[NBB];
  acc1[0] = acc1[1] = f4_t{0, 0, 0, 0};
#pragma unroll
  for (int bb = 0; bb < NBB; ++bb) acc2[bb] = f4_t{0, 0, 0, 0};
  const __bf16 *wrow = Wt + (16 * cb + r) * ldk + 8 * q;
  const __bf16 *yfrag = Ys + r * YR + 8 * q;
  const bool cb_live = NCB == 4 || 16 * cb < (int)p.L1;  // as in wfuse_kernel
  const int nbw = (int)((p.ipg + ULN - 1) / ULN) * bpu;
  int g = 0;
  for (int u = 0; u * bpu < nbw; ++u) {
    for (int bi = 0; bi < bpu; ++bi, ++g) {
      const int b = g & 1;
      if (b == 0) loady(g + 2, yr[0]); else loady(g + 2, yr[1]);
      static_for<0, NCB>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const int c = bi * NCB + s;
        if (c < nch && cb_live) {
          const bf8_t w = *reinterpret_cast<const bf8_t *>(wrow + 32 * c);
          const bf8_t y = *reinterpret_cast<const bf8_t *>(yfrag + (b * NCB + s) * POS);
          acc1[s & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, y, acc1[s & 1], 0, 0, 0);
        }
      });
      if (b == 0) stagey(1, yr[1]); else stagey(0, yr[0]);
      __syncthreads();
    }
    const f4_t zs = acc1[0] + acc1[1];
    acc1[0] = acc1[1] = f4_t{0, 0, 0, 0};
    const float zv[4] = {zs[0], zs[1], zs[2], zs[3]};
    const bf8_t z = bf16_lo4(zv);
    if constexpr (NCB == 4) {
#pragma unroll
      for (int bb = 0; bb < NBB; ++bb)
        acc2[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(z, bf16_lo4(sk[bb]), acc2[bb], 0, 0, 0);
    } else if (cb_live) {
#pragma unroll
      for (int bb = 0; bb < NBB; ++bb)
        if (bb < p.nbb)
          acc2[bb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(z, bf16_lo4(sk[bb]), acc2[bb], 0, 0, 0);
    }
    loadsk(u + 1, sk);
  }

  __syncthreads();
  float *red = reinterpret_cast<float *>(wf_lds);
  const int ncol = 16 * p.nbb;
#pragma unroll
  for (int bb = 0; bb < NBB; ++bb)
    if (bb < p.nbb) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) red[(wave * 16 + 4 * q + jj) * ncol + 16 * bb + r] = acc2[bb][jj];
    }
  __syncthreads();
  const int waves = blockDim.x >> 6;
  float *out = static_cast<float *>(ent.out);
  for (int e = tid; e < 16 * p.L0; e += blockDim.x) {
    const int rr = e / (int)p.L0, col = e - rr * (int)p.L0;
    const int64_t a = a0 + rr;
    if (a >= R0) continue;
    float acc = 0.f;
    for (int w = 0; w < waves; ++w) acc += red[(w * 16 + rr) * ncol + col];
    if (p.direct)
      out[a * p.L0 + col] = acc;
    else
      out[(grp * R0 + a) * p.L0 + col] = acc;
  }
}

// Sum of the i-range splits of every summand of a launch, in split order:
// W_(n-1)(a, b) = sum_g split_g(a, b).  blockIdx.y is the summand.
struct WSumEntry {
  const void *part;
  void *out;
  int64_t elems;  // R0 * L0
};
struct WSumArgs {
  int64_t groups;
  int count;
  WSumEntry e[kFuseMaxGroup];
};

template <typename T>
__global__ __launch_bounds__(256) void wfuse_sum_kernel(const WSumArgs a) {
  const WSumEntry &e = a.e[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= e.elems) return;
  const T *part = static_cast<const T *>(e.part);
  T acc = part[idx];
  for (int64_t g = 1; g < a.groups; ++g) acc += part[g * e.elems + idx];
  static_cast<T *>(e.out)[idx] = acc;
}

// gfx950: 160 KiB of LDS per workgroup, 256 CUs
constexpr size_t kMaxLds = 160 * 1024;
constexpr int kCUs = 256;

struct WFusePlan {
  WFuseArgs a{};
  int64_t groups = 1, tiles = 0;
  int64_t part_elems = 0;  // splits of all summands of the launch
  size_t lds = 0;
  int threads = 0;
  int nbb_t = 4;
};

// Plan of one launch over items [b, e) of the level.
bool plan(const WFuse &f, size_t b, size_t e, WFusePlan &pl) {
  const bool bf = f.math == DType::BF16;
  if (bf) {
    if (f.t != DType::F32 || (f.sk != DType::BF16 && f.sk != DType::F32)) return false;
  } else {
    if ((f.t != DType::F64 && f.t != DType::F32) || f.math != f.t || f.sk != f.t) return false;
  }
  if (e <= b || e - b > (size_t)kFuseMaxGroup) return false;
  if (f.I <= 0 || f.L1 <= 0 || f.L0 <= 0) return false;
  if (f.L1 > 128 || f.L0 > 128) return false;
  const size_t es = f.t == DType::F64 ? 8 : 4;  // storage of Y, W, C
  const size_t ss = f.sk == DType::BF16 ? 2 : es;  // storage of the sketch
  // staged values in LDS: the arithmetic type
  const size_t ls = bf ? 2 : es;
  const int kc = bf ? 32 : 16;  // k per position
  // buffer loads address Y, Sk_n and W_n with 32-bit offsets below 2^31
  if ((double)f.L0 * f.I * f.L1 * ss >= 2147483648.0) return false;
  int64_t r1max = 0;
  for (size_t k = b; k < e; ++k) {
    const WFuseItem &it = f.items[k];
    if (it.R0 <= 0 || it.R1 <= 0) return false;
    if (it.R1 % 4 != 0) return false;  // Y fragments are whole 4-vectors
    if ((double)it.R0 * f.I * it.R1 * es >= 2147483648.0) return false;
    if ((double)it.R1 * f.L1 * es >= 2147483648.0) return false;
    r1max = std::max(r1max, it.R1);
  }
  WFuseArgs &a = pl.a;
  a.I = f.I;
  a.L1 = f.L1;
  a.L0 = f.L0;
  // c-blocks padded to 4 (L1 <= 64) or 8, b-blocks to 4 or 8
  a.ncb = f.L1 <= 64 ? 4 : 8;
  a.nbb = (int)((f.L0 + 15) / 16);
  pl.nbb_t = a.nbb <= 4 ? 4 : 8;
  // row padding of W^T and of the staged Y: one 16-byte step per row spreads
  // the rows of a fragment read over the LDS banks; rows stay 16-byte aligned
  const int pad = (int)(16 / ls);
  const int64_t ldk_max = kc * ((r1max + kc - 1) / kc) + pad;
  const size_t ypos = (size_t)16 * (kc + pad);  // one staged Y position
  // unit lanes: as many as the registers allow (f64: three wavefronts per
  // SIMD for four c- and four b-blocks, else two; f32 and bf16: four), fewer
  // if the LDS cannot hold the staged Y of all lanes
  static const int kF64Ulns44[] = {3, 2, 1}, kF64Ulns48[] = {2, 1}, kF64Ulns8[] = {1},
                   kF32Ulns4[] = {4, 2, 1}, kF32Ulns8[] = {2, 1}, kBfUlns[] = {4, 2, 1};
  const int *ulns;
  int nulns;
  if (bf) {
    // one size per shape: 16 wavefronts, 8 with eight b-blocks
    ulns = kBfUlns + (a.ncb == 4 ? 0 : 1) + (pl.nbb_t == 4 ? 0 : 1);
    nulns = 1;
  } else if (f.t == DType::F64) {
    if (a.ncb == 4 && pl.nbb_t == 4) ulns = kF64Ulns44, nulns = 3;
    else if (a.ncb == 4) ulns = kF64Ulns48, nulns = 2;
    else ulns = kF64Ulns8, nulns = 1;
  } else {
    if (a.ncb == 4) ulns = kF32Ulns4, nulns = 3;
    else ulns = kF32Ulns8, nulns = 2;
  }
  const size_t acc_bytes = f.t == DType::F64 ? 8 : 4;
  int uln = 0;
  for (int k = 0; k < nulns && !uln; ++k) {
    const int u = ulns[k], waves = a.ncb * u;
    const size_t stage = ((size_t)16 * a.ncb * ldk_max + (size_t)u * 2 * a.ncb * ypos) * ls;
    const size_t red = (size_t)waves * 16 * 16 * a.nbb * acc_bytes;
    pl.lds = std::max(stage, red);
    if (pl.lds <= kMaxLds) uln = u;
  }
  if (!uln) return false;
  a.uln = uln;
  const int waves = a.ncb * uln;
  pl.threads = 64 * waves;
  // i-ranges: one count for all summands, about one wave of workgroups
  int64_t nablk = 0;
  for (size_t k = b; k < e; ++k) nablk += (f.items[k].R0 + 15) / 16;
  // wavefronts per CU the registers allow
  const int cap = bf ? (pl.nbb_t == 4 ? 16 : 12) : f.t == DType::F64 ? (uln == 3 ? 12 : 8) : 16;
  const int64_t per_cu = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)(kMaxLds / pl.lds), cap / waves));
  // at most 256 i-ranges
  int64_t g = std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(f.I, 256), kCUs * per_cu / nablk));
  a.ipg = (f.I + g - 1) / g;
  g = (f.I + a.ipg - 1) / a.ipg;
  pl.groups = g;
  a.direct = g == 1;
  a.count = (int)(e - b);
  int64_t tile = 0, part = 0;
  for (size_t k = b; k < e; ++k) {
    const WFuseItem &it = f.items[k];
    WFuseEntry &en = a.e[k - b];
    en.R0 = (int32_t)it.R0;
    en.R1 = (int32_t)it.R1;
    en.nch = (int32_t)((it.R1 + kc - 1) / kc);
    en.ldk = kc * en.nch + pad;
    en.nablk = (int32_t)((it.R0 + 15) / 16);
    en.tile0 = (int32_t)tile;
    tile += (int64_t)en.nablk * g;
    part += g == 1 ? 0 : g * it.R0 * f.L0;
  }
  pl.tiles = tile;
  pl.part_elems = part;
  return true;
}

template <int NCB, int NBB, int ULN, bool VS, typename TS>
int launch_bf16(const WFusePlan &pl, hipStream_t s) {
  static bool attr = false;
  if (!attr && pl.lds > 64 * 1024) {
    TTR_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void *>(&wfuse_bf16_kernel<NCB, NBB, ULN, VS, TS>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    attr = true;
  }
  const dim3 gr((unsigned)pl.tiles), bl((unsigned)pl.threads);
  hipLaunchKernelGGL((wfuse_bf16_kernel<NCB, NBB, ULN, VS, TS>), gr, bl, pl.lds, s, pl.a);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <int NCB, int NBB, int ULN, typename TS>
int launch_bf16_vs(const WFusePlan &pl, bool vs, hipStream_t s) {
  return vs ? launch_bf16<NCB, NBB, ULN, true, TS>(pl, s) : launch_bf16<NCB, NBB, ULN, false, TS>(pl, s);
}

template <typename TS>
int dispatch_bf16(const WFusePlan &pl, bool vs, hipStream_t s) {
  if (pl.a.ncb == 4)
    return pl.nbb_t == 4 ? launch_bf16_vs<4, 4, 4, TS>(pl, vs, s) : launch_bf16_vs<4, 8, 2, TS>(pl, vs, s);
  return pl.nbb_t == 4 ? launch_bf16_vs<8, 4, 2, TS>(pl, vs, s) : launch_bf16_vs<8, 8, 1, TS>(pl, vs, s);
}

template <class F, int NCB, int NBB, int ULN, bool VS>
int launch(const WFusePlan &pl, hipStream_t s) {
  static bool attr = false;
  if (!attr && pl.lds > 64 * 1024) {
    // dynamic LDS above 64 KiB is opted into once per kernel
    TTR_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&wfuse_kernel<F, NCB, NBB, ULN, VS>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    attr = true;
  }
  const dim3 gr((unsigned)pl.tiles), bl((unsigned)pl.threads);
  hipLaunchKernelGGL((wfuse_kernel<F, NCB, NBB, ULN, VS>), gr, bl, pl.lds, s, pl.a);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

// the unit-lane counts built for each shape (see plan)
template <class F, int NCB, int NBB, int ULN>
constexpr bool built() {
  if (std::is_same<F, FuseF64>::value)
    return NCB == 4 ? (NBB == 4 ? ULN <= 3 : ULN <= 2) : ULN == 1;
  return NCB == 4 ? (ULN == 1 || ULN == 2 || ULN == 4) : ULN <= 2;
}

template <class F, int NCB, int NBB, int ULN>
int launch_vs(const WFusePlan &pl, bool vs, hipStream_t s) {
  if constexpr (built<F, NCB, NBB, ULN>())
    return vs ? launch<F, NCB, NBB, ULN, true>(pl, s) : launch<F, NCB, NBB, ULN, false>(pl, s);
  return fail(TT_EINVAL, "internal: fused W-chain shape not built");
}

template <class F, int NCB, int NBB>
int dispatch_uln(const WFusePlan &pl, bool vs, hipStream_t s) {
  switch (pl.a.uln) {
    case 1: return launch_vs<F, NCB, NBB, 1>(pl, vs, s);
    case 2: return launch_vs<F, NCB, NBB, 2>(pl, vs, s);
    case 3: return launch_vs<F, NCB, NBB, 3>(pl, vs, s);
    default: return launch_vs<F, NCB, NBB, 4>(pl, vs, s);
  }
}

template <class F>
int dispatch_fuse(const WFusePlan &pl, bool vs, hipStream_t s) {
  if (pl.a.ncb == 4)
    return pl.nbb_t == 4 ? dispatch_uln<F, 4, 4>(pl, vs, s) : dispatch_uln<F, 4, 8>(pl, vs, s);
  return pl.nbb_t == 4 ? dispatch_uln<F, 8, 4>(pl, vs, s) : dispatch_uln<F, 8, 8>(pl, vs, s);
}

size_t elem_bytes(const WFuse &f) { return f.t == DType::F64 ? 8 : 4; }

}  // namespace

bool wfuse_supported(const WFuse &f) {
  WFusePlan pl;
  for (size_t b = 0; b < f.items.size(); b += kFuseMaxGroup)
    if (!plan(f, b, std::min(f.items.size(), b + kFuseMaxGroup), pl)) return false;
  return !f.items.empty();
}

int64_t wfuse_partial_elems(const WFuse &f) {
  // every launch of up to kFuseMaxGroup summands has its own part of the
  // buffer, so that all the splits can be summed after all the launches
  int64_t need = 0;
  WFusePlan pl;
  for (size_t b = 0; b < f.items.size(); b += kFuseMaxGroup)
    if (plan(f, b, std::min(f.items.size(), b + kFuseMaxGroup), pl)) need += pl.part_elems;
  return need;
}

bool wfuse_aligned(const WFuse &f) {
  for (const WFuseItem &it : f.items)
    if (reinterpret_cast<uintptr_t>(it.Y) % 16 != 0) return false;
  return true;
}

// splits of summand k: after those of every earlier summand of the level
int wfuse_run(const WFuse &f, void *partial, size_t partial_bytes, hipStream_t s) {
  if (!wfuse_aligned(f)) return fail(TT_EINVAL, "internal: fused W chain needs 16-byte aligned cores");
  const size_t es = elem_bytes(f);
  if ((size_t)wfuse_partial_elems(f) * es > partial_bytes || (!partial && partial_bytes == 0 &&
                                                               wfuse_partial_elems(f) > 0))
    return fail(TT_EINVAL, "internal: split buffer too small for the fused W chain");
  // Sk_n fragments as 4-vectors when its rows keep that alignment
  const size_t ss = f.sk == DType::BF16 ? 2 : es;
  const bool vs = f.L1 % 4 == 0 && reinterpret_cast<uintptr_t>(f.Sk) % (4 * ss) == 0;
  int64_t part = 0;
  for (size_t b = 0; b < f.items.size(); b += kFuseMaxGroup) {
    const size_t e = std::min(f.items.size(), b + kFuseMaxGroup);
    WFusePlan pl;
    if (!plan(f, b, e, pl)) return fail(TT_EINVAL, "internal: fused W-chain level not supported");
    WFuseArgs &a = pl.a;
    a.Sk = f.Sk;
    for (size_t k = b; k < e; ++k) {
      WFuseEntry &en = a.e[k - b];
      en.Y = f.items[k].Y;
      en.W = f.items[k].W;
      en.out = a.direct ? f.items[k].C : static_cast<char *>(partial) + part * es;
      if (!a.direct) part += pl.groups * f.items[k].R0 * f.L0;
    }
    if (f.math == DType::BF16)
      TTR_TRY(f.sk == DType::BF16 ? dispatch_bf16<__bf16>(pl, vs, s) : dispatch_bf16<float>(pl, vs, s));
    else
      TTR_TRY(f.t == DType::F64 ? dispatch_fuse<FuseF64>(pl, vs, s) : dispatch_fuse<FuseF32>(pl, vs, s));
  }
  return TT_OK;
}

int wfuse_sum(const WFuse &f, void *partial, hipStream_t s) {
  const size_t es = elem_bytes(f);
  int64_t part = 0;
  for (size_t b = 0; b < f.items.size(); b += kFuseMaxGroup) {
    const size_t e = std::min(f.items.size(), b + kFuseMaxGroup);
    WFusePlan pl;
    if (!plan(f, b, e, pl)) return fail(TT_EINVAL, "internal: fused W-chain level not supported");
    if (pl.a.direct) continue;
    WSumArgs sa{};
    sa.groups = pl.groups;
    sa.count = (int)(e - b);
    int64_t maxe = 0;
    for (size_t k = b; k < e; ++k) {
      WSumEntry &se = sa.e[k - b];
      se.part = static_cast<char *>(partial) + part * es;
      se.out = f.items[k].C;
      se.elems = f.items[k].R0 * f.L0;
      maxe = std::max(maxe, se.elems);
      part += pl.groups * se.elems;
    }
    const dim3 gr((unsigned)((maxe + 255) / 256), (unsigned)sa.count), bl(256);
    if (f.t == DType::F64)
      hipLaunchKernelGGL((wfuse_sum_kernel<double>), gr, bl, 0, s, sa);
    else
      hipLaunchKernelGGL((wfuse_sum_kernel<float>), gr, bl, 0, s, sa);
    TTR_HIP(hipGetLastError());
  }
  return TT_OK;
}

}  // namespace ttr
