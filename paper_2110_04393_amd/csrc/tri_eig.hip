// Leading eigenpairs of a small symmetric matrix with a short dependency
// chain, for the truncation step of the rounding.
//
// The truncation of the left-orthogonal RtO output (section 3.2, remark after
// Algorithm 5; the mirror of the truncation loop of Algorithm 2) diagonalises
// at every bond the Gram G = H(X_n) H(X_n)^T (n <= 76 here) and keeps its k
// leading eigenpairs.  On a GPU the cost of such a solve is the length of its
// chain of dependent steps, so the method is chosen for that:
//
//   1. Householder tridiagonalisation G = Q T Q^T with the matrix in
//      registers (tri_reduce_kernel, one workgroup, two barriers per column;
//      the reflectors are kept for step 3, with the products v_j^T v_(j+1)
//      and v_j^T v_(j+2)).
//   2. The k+1 leading eigenvalues (the (k+1)-th to check the gap) by
//      multisection, one wavefront per eigenvalue (tri_vec_kernel): the 64
//      lanes evaluate Sturm counts at 64 points of the bracket (65-fold
//      shrink, 9 iterations), each count the sign changes of the
//      leading-minor determinants p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}
//      (one dependent FMA per step, rescaled by powers of two).
//   3. In the same wavefront, the eigenvector of T by twisted factorisation
//      (T - lambda I = L+ D+ L+^T = U- D- U-^T, pivots as ratios of
//      consecutive minors; twist r = argmin |gamma_r|; z_r = 1 and z
//      propagated outwards with the factors), then u = Q z with the
//      reflectors of step 1 applied three at a time.
//   4. tri_finish_kernel: one Newton-Schulz step Z <- Z (3/2 I - 1/2 Z^T Z)
//      (FP64 MFMA products in LDS) restores orthogonality lost to close
//      eigenvalues, then the factors of the truncation.
//
// The finish kernel runs the cyclic Jacobi solver (jacobi.h) itself instead
// when the wanted eigenvalues are not separated by 1e-9 ||T|| (repeated or
// near-repeated eigenvalues, an exactly split T) or the orthogonality defect
// before the Newton-Schulz step exceeds 1e-6.
#include "fastmath.h"
#include "jacobi.h"
#include "ldsmm.h"
#include "tt_internal.h"
#include "wave.h"

namespace ttr {
namespace {

constexpr int kTeThreads = 1024;
constexpr int kTeNMax = 76;

// ---------------------------------------------------------------- DPP
// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140
__device__ __forceinline__ double sum8(double v) {
  v += dppd<0xB1>(v);
  v += dppd<0x4E>(v);
  v += dppd<0x141>(v);
  return v;
}
__device__ __forceinline__ double sum16(double v) {
  v = sum8(v);
  return v + dppd<0x140>(v);
}
__device__ __forceinline__ double max16(double v) {
  v = fmax(v, dppd<0xB1>(v));
  v = fmax(v, dppd<0x4E>(v));
  v = fmax(v, dppd<0x141>(v));
  return fmax(v, dppd<0x140>(v));
}
__device__ __forceinline__ double min16(double v) {
  v = fmin(v, dppd<0xB1>(v));
  v = fmin(v, dppd<0x4E>(v));
  v = fmin(v, dppd<0x141>(v));
  return fmin(v, dppd<0x140>(v));
}
__device__ __forceinline__ double max8(double v) {
  v = fmax(v, dppd<0xB1>(v));
  v = fmax(v, dppd<0x4E>(v));
  return fmax(v, dppd<0x141>(v));
}
__device__ __forceinline__ double min8(double v) {
  v = fmin(v, dppd<0xB1>(v));
  v = fmin(v, dppd<0x4E>(v));
  return fmin(v, dppd<0x141>(v));
}
// Full-wavefront reductions, result uniform (all 64 lanes must be active).
// After the row reduction every lane of row r holds row r's result; row 1
// then combines row 0's (lane 15) and row 3 row 2's (lane 47), and rows 2
// and 3 combine lane 31's, so that lane 63 holds the result, in the order
// (r0 op r1) op (r2 op r3) for sums.  Rows 0 and 2 combine a 0 read from
// outside the broadcast in between, which never reaches lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v = sum16(v);
  v += dpp_row_bcast<0x142, 0xA>(v);
  v += dpp_row_bcast<0x143, 0xC>(v);
  return readlane_d(v, 63);
}
// two sums at once, their steps interleaved
__device__ __forceinline__ void wave_sum2(double &a, double &b) {
  a += dppd<0xB1>(a);
  b += dppd<0xB1>(b);
  a += dppd<0x4E>(a);
  b += dppd<0x4E>(b);
  a += dppd<0x141>(a);
  b += dppd<0x141>(b);
  a += dppd<0x140>(a);
  b += dppd<0x140>(b);
  a += dpp_row_bcast<0x142, 0xA>(a);
  b += dpp_row_bcast<0x142, 0xA>(b);
  a += dpp_row_bcast<0x143, 0xC>(a);
  b += dpp_row_bcast<0x143, 0xC>(b);
  a = readlane_d(a, 63);
  b = readlane_d(b, 63);
}
// three sums at once, their steps interleaved
__device__ __forceinline__ void wave_sum3(double &a, double &b, double &c) {
  a += dppd<0xB1>(a);
  b += dppd<0xB1>(b);
  c += dppd<0xB1>(c);
  a += dppd<0x4E>(a);
  b += dppd<0x4E>(b);
  c += dppd<0x4E>(c);
  a += dppd<0x141>(a);
  b += dppd<0x141>(b);
  c += dppd<0x141>(c);
  a += dppd<0x140>(a);
  b += dppd<0x140>(b);
  c += dppd<0x140>(c);
  a += dpp_row_bcast<0x142, 0xA>(a);
  b += dpp_row_bcast<0x142, 0xA>(b);
  c += dpp_row_bcast<0x142, 0xA>(c);
  a += dpp_row_bcast<0x143, 0xC>(a);
  b += dpp_row_bcast<0x143, 0xC>(b);
  c += dpp_row_bcast<0x143, 0xC>(c);
  a = readlane_d(a, 63);
  b = readlane_d(b, 63);
  c = readlane_d(c, 63);
}
__device__ __forceinline__ double wave_max(double v) {
  v = max16(v);
  v = fmax(v, dpp_row_bcast<0x142, 0xA>(v));
  v = fmax(v, dpp_row_bcast<0x143, 0xC>(v));
  return readlane_d(v, 63);
}
// the same for an int
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ int wave_min_int(int v) {
  v = min(v, dppi<0xB1>(v));
  v = min(v, dppi<0x4E>(v));
  v = min(v, dppi<0x141>(v));
  v = min(v, dppi<0x140>(v));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x142, 0xA, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x143, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ double wave_min(double v) {
  v = min16(v);
  v = fmin(v, dpp_row_bcast<0x142, 0xA>(v));
  v = fmin(v, dpp_row_bcast<0x143, 0xC>(v));
  return readlane_d(v, 63);
}


// ---------------------------------------------------------------- kernel 1
// Householder tridiagonalisation of the n x n symmetric Gin (n <= NMAX, one
// workgroup of four wavefronts, the matrix in registers).  Row i = 16 a + ty
// belongs to wavefront a % 4 and is spread over the lane quad 4 ty .. 4 ty + 3:
// lane tq holds the columns c = tq + 4 b.  The rank-2 update is two FMAs
// per entry, so the matrix stays symmetric to rounding only; the quad
// owning row j builds the reflector of step j from that row (an O(u ||A||)
// perturbation of the symmetric step, as the update's own rounding), and
// p = tau A v is a quad reduction within the owners of each row.  Per
// column the wavefronts exchange v, then p and the partial sums of p^T v,
// through LDS: two barriers.  Writes the scaled d (n), e (n-1) with
// ||T|| sc <= 1, the scale sc, and the reflectors (Vr row j = v_j over rows
// j+1..n-1, v_j[0] = 1; taus[j]) to global scratch, followed in Vr by the
// products v_j^T v_(j+1) (j < n-3) and v_j^T v_(j+2) (j < n-4) with which
// the eigenvector kernel applies the reflectors three at a time.
constexpr int kTrThreads = 256;

// a - vi wc - wi vc (two FMAs)
__device__ __forceinline__ double sym_update(double a, double vi, double wc, double wi,
                                             double vc) {
  return fma(-vi, wc, fma(-wi, vc, a));
}

template <int NMAX>
__device__ __forceinline__ void tri_reduce_body(const double *Gin, int n, double *d_out,
                                                double *e_out, double *sc_out, double *Vr,
                                                double *taus, int *flag) {
  constexpr int NB = NMAX / 4;       // column slots per lane
  constexpr int NA = NMAX / 16;      // row blocks
  constexpr int NS = (NA + 3) / 4;   // row slots per lane
  // reflector j at s_V[j], p of step j at s_p[j & 1]; entry c at (c % 4) NB + c / 4.
  // The reflectors, taus, d and e reach global memory only after the loop:
  // a barrier waits for the workgroup's outstanding global stores.
  __shared__ double s_V[NMAX][NMAX], s_p[2][NMAX];
  __shared__ double s_q[2][4], s_tau[NMAX];
  __shared__ double s_d[NMAX], s_e[NMAX];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ty = lane >> 2, tq = lane & 3;

  double A[NS][NB];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int i = 16 * (wave + 4 * sl) + ty;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c = tq + 4 * b;
      A[sl][b] = (i < n && c < n) ? (i >= c ? Gin[i * n + c] : Gin[c * n + i]) : 0.0;
    }
  }
  if (n <= 2) {
    if (tid == 0) {
      s_d[0] = Gin[0];
      if (n == 2) {
        s_e[0] = Gin[n];
        s_d[1] = Gin[n + 1];
      }
    }
  }
  static_for<0, NMAX - 2>([&](auto jc) __attribute__((always_inline)) {
    constexpr int j = decltype(jc)::value;
    if (j > n - 3) return;
    constexpr int buf = j & 1;
    constexpr int js = (j / 16) / 4, jw = (j / 16) % 4;
    // ---- phase 1: the quad owning row j (= column j) builds the reflector
    if (wave == jw && ty == j % 16) {
      double sq[4] = {0.0, 0.0, 0.0, 0.0};  // four independent chains
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (4 * b + 3 >= j + 2) {
          const int c = tq + 4 * b;
          if (c >= j + 2) sq[b & 3] = fma(A[js][b], A[js][b], sq[b & 3]);
        }
      }
      const double sigma = quad_sum((sq[0] + sq[1]) + (sq[2] + sq[3]));
      const double a0 = quad_bcast<(j + 1) % 4>(A[js][(j + 1) / 4]);
      const double djj = quad_bcast<j % 4>(A[js][j / 4]);
      double beta, tau, scale;
      if (sigma == 0.0) {
        beta = a0;
        tau = 0.0;
        scale = 0.0;
      } else {
        const double mu = sqrt_f64(fma(a0, a0, sigma));
        beta = (a0 >= 0.0) ? -mu : mu;
        tau = (beta - a0) * rcp_f64(beta);
        scale = rcp_f64(a0 - beta);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int c = tq + 4 * b;
        s_V[j][tq * NB + b] = (c == j + 1) ? 1.0 : ((c > j + 1) ? A[js][b] * scale : 0.0);
      }
      if (tq == 0) {
        s_tau[j] = tau;
        s_e[j] = beta;
        s_d[j] = djj;
      }
    }
    __syncthreads();
    // ---- phase 2: p = tau A v (rows of this lane quad), partial p^T v
    const double tau = s_tau[j];
    double vc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) vc[b] = s_V[j][tq * NB + b];
    double vr[NS], pr[NS];
    double qpart = 0.0;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int i = 16 * (wave + 4 * sl) + ty;
      vr[sl] = 0.0;
      pr[sl] = 0.0;
      if (16 * (wave + 4 * sl) + 15 > j && 16 * (wave + 4 * sl) < NMAX) {
        vr[sl] = s_V[j][(i & 3) * NB + (i >> 2)];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (4 * b + 3 > j) acc[b & 3] = fma(A[sl][b], vc[b], acc[b & 3]);
        pr[sl] = tau * quad_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
        if (tq == 0) {
          s_p[buf][(i & 3) * NB + (i >> 2)] = pr[sl];
          qpart = fma(pr[sl], vr[sl], qpart);
        }
      }
    }
    const double qw = wave_sum(qpart);
    if (lane == 0) s_q[buf][wave] = qw;
    __syncthreads();
    // ---- phase 3: w = p - K v, A -= v w^T + w v^T on the live part
    const double K = 0.5 * tau * ((s_q[buf][0] + s_q[buf][1]) + (s_q[buf][2] + s_q[buf][3]));
    double wc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) wc[b] = (4 * b + 3 > j) ? s_p[buf][tq * NB + b] - K * vc[b] : 0.0;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      if (16 * (wave + 4 * sl) + 15 > j && 16 * (wave + 4 * sl) < NMAX) {
        const double wr = pr[sl] - K * vr[sl];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (4 * b + 3 > j) A[sl][b] = sym_update(A[sl][b], vr[sl], wc[b], wr, vc[b]);
      }
    }
    if (j == n - 3) {
      // the trailing 2 x 2 block: rows j+1 and j+2
      constexpr int r1 = j + 1, r2 = j + 2;
      if (wave == (r1 / 16) % 4 && ty == r1 % 16) {
        const double dd = quad_bcast<(j + 1) % 4>(A[(r1 / 16) / 4][(j + 1) / 4]);
        const double ee = quad_bcast<(j + 2) % 4>(A[(r1 / 16) / 4][(j + 2) / 4]);
        if (tq == 0) {
          s_d[r1] = dd;
          s_e[r1] = ee;
        }
      }
      if (wave == (r2 / 16) % 4 && ty == r2 % 16) {
        const double dd = quad_bcast<(j + 2) % 4>(A[(r2 / 16) / 4][(j + 2) / 4]);
        if (tq == 0) s_d[r2] = dd;
      }
    }
  });
  __syncthreads();
  // reflectors (Vr row j = v_j over rows j+1..n-1) and taus
  for (int e = tid; e < (n - 2) * n; e += kTrThreads) {
    const int j = e / n, r = e - j * n, c = r + j + 1;
    if (c < n) Vr[e] = s_V[j][(c & 3) * NB + (c >> 2)];
  }
  for (int j = tid; j < n - 2; j += kTrThreads) taus[j] = s_tau[j];
  // v_j^T v_(j+1) (v_(j+1) starts at row j + 2) and v_j^T v_(j+2) (row j + 3)
  for (int t = tid; t < 2 * n - 7; t += kTrThreads) {
    const int dist = t < n - 3 ? 1 : 2, j = t < n - 3 ? t : t - (n - 3);
    double acc = 0.0;
    for (int c = j + 1 + dist; c < n; ++c)
      acc = fma(s_V[j][(c & 3) * NB + (c >> 2)], s_V[j + dist][(c & 3) * NB + (c >> 2)], acc);
    Vr[(n - 2) * n + t] = acc;
  }
  if (wave == 0) {
    double mx = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double rad = (i > 0 ? fabs(s_e[i - 1]) : 0.0) + (i < n - 1 ? fabs(s_e[i]) : 0.0);
      mx = fmax(mx, fabs(s_d[i]) + rad);
    }
    mx = wave_max(mx);
    const double sc = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ilogb(mx) - 1) : 1.0;
    for (int i = lane; i < n; i += 64) {
      d_out[i] = s_d[i] * sc;
      if (i < n - 1) e_out[i] = s_e[i] * sc;
    }
    if (lane == 0) {
      *sc_out = sc;
      *flag = (mx > 0.0 && isfinite(mx)) ? 0 : 1;
    }
  }
}

template <int NMAX>
__global__ __launch_bounds__(kTrThreads) void tri_reduce_kernel(const double *Gin, int n,
                                                                double *d_out, double *e_out,
                                                                double *sc_out, double *Vr,
                                                                double *taus, int *flag) {
  tri_reduce_body<NMAX>(Gin, n, d_out, e_out, sc_out, Vr, taus, flag);
}

// ---------------------------------------------------------------- kernel 2
// One wavefront per wanted eigenvalue w (descending, w < kw).  T (n <= NMAX)
// is staged in LDS and padded to NMAX with d = 4, e = 0: T is scaled to
// ||T|| <= 1, so the padding only adds eigenvalues at 4, outside every
// bracket, and every recurrence runs a fixed, unrolled number of steps
// without branches.
//  * eigenvalue: 64-point multisection of [-1, 1] (9 iterations of a 65-fold
//    shrink); lane l counts the sign changes of the leading-minor
//    determinants p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2} at its point,
//    rescaled by a power of two every 8 steps, one FMA per step on the
//    dependent chain.  An exact zero p_i counts by its sign bit (+0 as
//    positive): then p_{i+1} = -e_i^2 p_{i-1} has the sign opposite to
//    p_{i-1}, so the two changes p_{i-1} -> p_i -> p_{i+1} count one whatever
//    sign p_i is given, as in the usual convention; only a zero as the last
//    minor (x itself an eigenvalue) may count differently, which moves x to
//    one side of the bracket without changing the limit;
//  * for w < k the eigenvector: twisted factorisation (lanes 0-31 the
//    top-down LDL^T, lanes 32-63 the same recurrence on the reversed matrix,
//    i.e. the bottom-up UDU^T; pivots as ratios of consecutive minors, so the
//    chain is one FMA per step), twist r = argmin |gamma_r|, z from products
//    of the factors (log-step scans), then the Householder reflectors of
//    kernel 1 applied backwards give u = Q z, written to column w of U (n x k)
//    unnormalised by sc.  The reflectors go three at a time: for H_a H_b H_c
//    (a = b - 1 = c - 2, c applied first) the products v_c^T z, v_b^T z,
//    v_a^T z are reduced together, and the updates they miss follow from the
//    products of the reflectors themselves (from kernel 1): v_b^T (H_c z) =
//    v_b^T z - tau_c (v_b^T v_c) (v_c^T z), and so on, so the chain holds
//    one wavefront reduction per block.
constexpr double kTiny = 1e-300;

template <int NMAX>
__device__ __forceinline__ void tri_vec_body(const double *d_in, const double *e_in, int n, int k,
                                             const double *Vr, const double *taus,
                                             double *lam_out, double *Uz, const int *flag,
                                             int w) {
  if (*flag) return;
  __shared__ double s_d[NMAX + 1], s_e[NMAX + 1], s_e2[NMAX + 1];
  __shared__ double s_dr[NMAX + 1], s_er[NMAX + 1], s_er2[NMAX + 1];  // T reversed
  __shared__ double2 s_pq[2 * NMAX];  // (p_i, p_{i-1}) of both directions
  __shared__ double2 s_pqj[8 * 64];    // the other lanes' copies
  __shared__ double s_f[2][NMAX];  // L_i (top-down), U_{n-1-i} (bottom-up)
  __shared__ double s_z[NMAX];
  __shared__ double s_V[NMAX * NMAX + 1];  // reflectors: s_V[j n + i - j - 1]; last: 0
  __shared__ double s_tau[NMAX], s_vv[NMAX], s_vv2[NMAX];  // tau_j, v_j^T v_(j+1), v_j^T v_(j+2)
  __shared__ double s_sc[2][2][128];   // scan buffers (lower, upper factors)
  const int lane = threadIdx.x;
  if (n >= 5) {
    // every load first, all in flight together (indices clamped into d_in
    // (n), e_in (n - 1), taus (n - 2) and Vr (n^2); values outside the
    // ranges below are dropped), then the LDS stores
    constexpr int NI = (NMAX + 1 + 63) / 64, NJ = (NMAX + 63) / 64;
    double dv[NI], ev[NI], drv[NI], erv[NI], tv[NJ], v1[NJ], v2[NJ];
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int i = lane + 64 * u;
      dv[u] = d_in[min(i, n - 1)];
      ev[u] = e_in[min(i, n - 2)];
      drv[u] = d_in[max(n - 1 - i, 0)];
      erv[u] = e_in[max(n - 2 - i, 0)];
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = lane + 64 * u;
      tv[u] = taus[min(j, n - 3)];
      v1[u] = Vr[(n - 2) * n + min(j, n - 4)];
      v2[u] = Vr[(n - 2) * n + (n - 3) + min(j, n - 5)];
    }
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int i = lane + 64 * u;
      if (i <= NMAX) {
        const double d = (i < n) ? dv[u] : 4.0, e = (i < n - 1) ? ev[u] : 0.0;
        const double er = (i < n - 1) ? erv[u] : 0.0;
        s_d[i] = d;
        s_e[i] = e;
        s_e2[i] = e * e;
        s_dr[i] = (i < n) ? drv[u] : 4.0;
        s_er[i] = er;
        s_er2[i] = er * er;
      }
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = lane + 64 * u;
      if (j < n - 2) s_tau[j] = tv[u];
      if (j < n - 3) s_vv[j] = v1[u];
      if (j < n - 4) s_vv2[j] = v2[u];
    }
  } else {
    for (int i = lane; i <= NMAX; i += 64) {
      const double dv = (i < n) ? d_in[i] : 4.0;
      const double ev = (i < n - 1) ? e_in[i] : 0.0;
      s_d[i] = dv;
      s_e[i] = ev;
      s_e2[i] = ev * ev;
      s_dr[i] = (i < n) ? d_in[n - 1 - i] : 4.0;
      s_er[i] = (i < n - 1) ? e_in[n - 2 - i] : 0.0;
      s_er2[i] = s_er[i] * s_er[i];
    }
    for (int j = lane; j < n - 2; j += 64) s_tau[j] = taus[j];
    for (int j = lane; j < n - 3; j += 64) s_vv[j] = Vr[(n - 2) * n + j];
    for (int j = lane; j < n - 4; j += 64) s_vv2[j] = Vr[(n - 2) * n + (n - 3) + j];
  }
  if (lane == 0) s_V[NMAX * NMAX] = 0.0;
  __syncthreads();
  // The reflectors go from global memory straight to LDS (16 bytes per lane
  // and load, no registers) while the eigenvalue and the twisted
  // factorisation run, which do not read them; the barrier after the
  // factorisation waits for the loads.  Only the waves that form an
  // eigenvector load them (and so never end with a load in flight).  A lane
  // loads the pair e, e + 1 with e < total <= n^2 - 2, inside Vr's n^2 values.
  if (w < k) {
    const int total = (n - 2) * n;
    for (int e0 = 0; e0 < total; e0 += 128)
      if (e0 + 2 * lane < total)
        __builtin_amdgcn_global_load_lds(
            static_cast<const void *>(Vr + e0 + 2 * lane),
            (__attribute__((address_space(3))) void *)(s_V + e0), 16, 0, 0);
  }

  const int a = n - 1 - w;
  double lo = -1.0 - 1e-13, hi = 1.0 + 1e-13;
  for (int it = 0; it < 9; ++it) {
    const double x = lo + (double)(lane + 1) * (hi - lo) * (1.0 / 65.0);
    double pp = 1.0, p = s_d[0] - x;
    int cnt = (int)((unsigned)__double2hiint(p) >> 31);
    static_for<1, NMAX>([&](auto ic) __attribute__((always_inline)) {
      constexpr int i = decltype(ic)::value;
      const double pn = fma(s_d[i] - x, p, -s_e2[i - 1] * pp);
      cnt += (int)((unsigned)(__double2hiint(pn) ^ __double2hiint(p)) >> 31);
      pp = p;
      p = pn;
      if constexpr (i % 8 == 0) {
        const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(p), fabs(pp)));
        p = ldexp(p, -ex);
        pp = ldexp(pp, -ex);
      }
    });
    const double cl = (cnt <= a) ? x : lo;
    const double ch = (cnt > a) ? x : hi;
    lo = wave_max(cl);
    hi = wave_min(ch);
  }
  const double lam = 0.5 * (lo + hi);
  if (lane == 0) lam_out[w] = lam;
  if (w >= k) return;
  // twisted factorisation: lanes 0-31 run the top-down recurrence on T, lanes
  // 32-63 on T reversed; lane 0 gives L_i, lane 32 gives U_{n-1-i}.  The
  // pivots D_i = (d_i - lam) - e_{i-1}^2 / D_{i-1} are the ratios p_i / p_{i-1}
  // of the leading minors of T - lam I, p_i = (d_i - lam) p_{i-1} -
  // e_{i-1}^2 p_{i-2}: the chain runs that recurrence (one FMA per step, with
  // the same relative perturbations of d_i - lam, e^2 and the result per step
  // as the pivot recurrence), the writer keeps each pair (p_i, p_{i-1}) in one
  // scale, and L_i = e_i / D_i = e_i p_{i-1} / p_i is formed afterwards for all
  // i at once (a zero pivot replaced by a tiny one, as in the pivot form).
  const bool rev = lane >= 32;
  {
    const double *D = rev ? s_dr : s_d;
    const double *E2 = rev ? s_er2 : s_e2;
    // lanes 0 and 32 write step i to slot i, the others to eight slots of
    // their own (one per step of a block): one store per step at a fixed
    // offset from a block base, and no branch in the chain
    const bool writer = (lane & 31) == 0;
    double2 *const PQ = writer ? s_pq + (rev ? NMAX : 0) : s_pqj + 8 * lane;
    double2 *blk = PQ;
    // d_{i+1} and e_i^2 in blocks of 8 steps, each block loaded one block ahead
    double dc[8], ec[8], dn[8], en[8];
    static_for<0, 8>([&](auto uc) __attribute__((always_inline)) {
      constexpr int u = decltype(uc)::value;
      dc[u] = D[u + 1];
      ec[u] = E2[u];
    });
    double pp = 1.0, p = D[0] - lam;
    static_for<0, NMAX - 1>([&](auto ic) __attribute__((always_inline)) {
      constexpr int i = decltype(ic)::value, t = i % 8;
      if constexpr (t == 0) {
        blk = writer ? PQ + i : PQ;
        static_for<0, 8>([&](auto uc) __attribute__((always_inline)) {
          constexpr int u = decltype(uc)::value, ii = i + 8 + u;
          if constexpr (ii < NMAX - 1) {
            dn[u] = D[ii + 1];
            en[u] = E2[ii];
          }
        });
      }
      blk[t] = make_double2(p, pp);
      const double pn = fma(dc[t] - lam, p, -ec[t] * pp);
      pp = p;
      p = pn;
      if constexpr (t == 7) {
        const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(p), fabs(pp)));
        p = ldexp(p, -ex);
        pp = ldexp(pp, -ex);
        static_for<0, 8>([&](auto uc) __attribute__((always_inline)) {
          constexpr int u = decltype(uc)::value;
          dc[u] = dn[u];
          ec[u] = en[u];
        });
      }
    });
  }
  __syncthreads();
  for (int i = lane; i < 2 * (NMAX - 1); i += 64) {
    const int h = i >= NMAX - 1 ? 1 : 0, t = i - h * (NMAX - 1);
    const double2 q = s_pq[h * NMAX + t];
    double dp = q.x * rcp_f64(q.y);
    if (dp == 0.0) dp = kTiny;
    s_f[h][t] = (h ? s_er[t] : s_e[t]) * rcp_f64(dp);
  }
  __syncthreads();
  // L_i = s_f[0][i], U_i = s_f[1][n-1-i]
  // gamma_i = delta_i - L_{i-1} e_{i-1} - U_{i+1} e_i, twist r = argmin |gamma|
  double best = 1e300;
  int rbest = 0;
  for (int i = lane; i < n; i += 64) {
    double g = s_d[i] - lam;
    if (i > 0) g -= s_f[0][i - 1] * s_e[i - 1];
    if (i < n - 1) g -= s_f[1][n - 2 - i] * s_e[i];
    g = fabs(g);
    if (g < best) {
      best = g;
      rbest = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int orr = __shfl_xor(rbest, off);
    if (ob < best || (ob == best && orr < rbest)) {
      best = ob;
      rbest = orr;
    }
  }
  const int r = rbest;
  // z_r = 1, z_i = prod_{k=i}^{r-1} (-L_k) below the twist and
  // prod_{k=r+1}^{i} (-U_k) above it: a suffix and a prefix product over
  // 128 slots (lane l holds slots l and l + 64), log-step scans through LDS
  {
    double lo_f[2], up_f[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      lo_f[h] = (i < r) ? -s_f[0][i] : 1.0;
      up_f[h] = (i > r && i < n) ? -s_f[1][n - 1 - i] : 1.0;
      s_sc[0][0][i] = lo_f[h];
      s_sc[0][1][i] = up_f[h];
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 7; ++st) {
      const int off = 1 << st, src = st & 1, dst = src ^ 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i + off < 128) lo_f[h] *= s_sc[src][0][i + off];
        if (i - off >= 0) up_f[h] *= s_sc[src][1][i - off];
        s_sc[dst][0][i] = lo_f[h];
        s_sc[dst][1][i] = up_f[h];
      }
      __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i < n) s_z[i] = (i < r) ? lo_f[h] : ((i > r) ? up_f[h] : 1.0);
    }
  }
  __syncthreads();
  // normalise, then u = H_0 H_1 ... H_{n-3} z (apply from the last reflector)
  double z0 = (lane < n) ? s_z[lane] : 0.0, z1 = (lane + 64 < n) ? s_z[lane + 64] : 0.0;
  const double inv = rsq_f64(wave_sum(z0 * z0 + z1 * z1));
  z0 *= inv;
  z1 *= inv;
  const int i0 = lane, i1 = lane + 64;
  // v_j at the rows of this lane: rows outside j+1..n-1 read the zero kept
  // after the reflectors, so every lane reads without a branch
  auto vrow = [&](int j, int i) -> double {
    return s_V[(i > j && i < n) ? j * n + i - j - 1 : NMAX * NMAX];
  };
  // blocks of three reflectors (c = j applied first, then b = j-1, a = j-2)
  int j = n - 3;
  for (; j >= 2; j -= 3) {
    const int c = j, b = j - 1, a = j - 2;
    const double vc0 = vrow(c, i0), vb0 = vrow(b, i0), va0 = vrow(a, i0);
    const double vc1 = NMAX > 64 ? vrow(c, i1) : 0.0, vb1 = NMAX > 64 ? vrow(b, i1) : 0.0;
    const double va1 = NMAX > 64 ? vrow(a, i1) : 0.0;
    double sc = fma(vc1, z1, vc0 * z0), sb = fma(vb1, z1, vb0 * z0), sa = fma(va1, z1, va0 * z0);
    wave_sum3(sc, sb, sa);
    const double cc = s_tau[c] * sc;
    const double cb = s_tau[b] * fma(-s_vv[b], cc, sb);
    const double ca = s_tau[a] * fma(-s_vv[a], cb, fma(-s_vv2[a], cc, sa));
    z0 = fma(-ca, va0, fma(-cb, vb0, fma(-cc, vc0, z0)));
    z1 = fma(-ca, va1, fma(-cb, vb1, fma(-cc, vc1, z1)));
  }
  if (j == 1) {
    const int b = 1, a = 0;
    const double vb0 = vrow(b, i0), va0 = vrow(a, i0);
    const double vb1 = NMAX > 64 ? vrow(b, i1) : 0.0, va1 = NMAX > 64 ? vrow(a, i1) : 0.0;
    double sb = fma(vb1, z1, vb0 * z0), sa = fma(va1, z1, va0 * z0);
    wave_sum2(sb, sa);
    const double cb = s_tau[b] * sb;
    const double ca = s_tau[a] * fma(-s_vv[a], cb, sa);
    z0 = fma(-ca, va0, fma(-cb, vb0, z0));
    z1 = fma(-ca, va1, fma(-cb, vb1, z1));
  } else if (j == 0) {
    const double v0 = vrow(0, i0), v1 = NMAX > 64 ? vrow(0, i1) : 0.0;
    const double c0 = s_tau[0] * wave_sum(fma(v1, z1, v0 * z0));
    z0 = fma(-c0, v0, z0);
    z1 = fma(-c0, v1, z1);
  }
  if (lane < n) Uz[lane * k + w] = z0;
  if (lane + 64 < n) Uz[(lane + 64) * k + w] = z1;
}

template <int NMAX>
__global__ __launch_bounds__(64) void tri_vec_kernel(const double *d_in, const double *e_in, int n,
                                                     int k, const double *Vr, const double *taus,
                                                     double *lam_out, double *Uz,
                                                     const int *flag) {
  tri_vec_body<NMAX>(d_in, e_in, n, k, Vr, taus, lam_out, Uz, flag, blockIdx.x);
}

// U1 (n x n, row-major, global) = [Z[:, :w] | C]: the w orthonormal columns
// of Z (LDS, leading dimension ld) and an orthonormal basis C of their
// complement (the basis of the second truncation pass, trunc_refine.hip).
// C comes from a pivoted Cholesky factorisation of the projector
// P = I - Z_w Z_w^T (rank n - w): P = C C^T with C of full column rank, so
// C = V Q for any orthonormal basis V of range(P) and an orthogonal Q, i.e.
// C has orthonormal columns itself; the diagonal pivoting keeps every step
// at a pivot of at least (n - w - j) / n of the remaining trace.  n - w steps
// of a rank-1 update, one barrier each: P alternates between Pa and Pb (LDS,
// n x ld each), every wavefront finds the pivot itself (largest diagonal
// entry, lowest index on ties) and every thread forms the entries of the
// pivot column it needs, so nothing is handed between wavefronts within a
// step.  All threads of the workgroup (at most kTeThreads).
__device__ void complement_basis(const double *Z, int ld, int n, int w, double *Pa, double *Pb,
                                 double *U1) {
  constexpr int kPer = (kTeNMax * kTeNMax + kTeThreads - 1) / kTeThreads;
  const int tid = threadIdx.x, lane = tid & 63;
  lds_gemm<false, true>(Z, ld, Z, ld, Pa, ld, n, n, w, -1.0, nullptr, 0, 0.0);
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) Pa[i * ld + i] += 1.0;
  for (int e = tid; e < n * w; e += blockDim.x) {
    const int i = e / w, c = e - i * w;
    U1[i * n + c] = Z[i * ld + c];
  }
  // the entries (i, c) of P this thread updates, the same at every step
  int ei[kPer], ec[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * kTeThreads;
    ei[u] = e < n * n ? e / n : -1;
    ec[u] = e < n * n ? e - (e / n) * n : 0;
  }
  __syncthreads();
  for (int j = 0; j < n - w; ++j) {
    const double d0 = lane < n ? Pa[lane * ld + lane] : -1e300;
    const double d1 = lane + 64 < n ? Pa[(lane + 64) * ld + lane + 64] : -1e300;
    const double best = fmax(d0, d1);
    const int bi = d1 > d0 ? lane + 64 : lane;
    const double mx = wave_max(best);
    const int pv = wave_min_int(best == mx ? bi : 1 << 30);
    const double rp = rsq_f64(fmax(mx, 1e-300));
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (ei[u] >= 0) {
        const int i = ei[u], c = ec[u];
        Pb[i * ld + c] = fma(-(Pa[i * ld + pv] * rp), Pa[c * ld + pv] * rp, Pa[i * ld + c]);
      }
    }
    for (int i = tid; i < n; i += blockDim.x) U1[i * n + w + j] = Pa[i * ld + pv] * rp;
    __syncthreads();
    double *t = Pa;
    Pa = Pb;
    Pb = t;
  }
}

// ---------------------------------------------------------------- kernel 3
// One workgroup: gap check, orthogonality check and one Newton-Schulz step on
// U (n x k, from kernel 2), outputs (unscaled eigenvalues, U, truncation
// factors, tail).
// Returns false (all threads alike, outputs untouched) when a check fails.
template <typename T>
__device__ __forceinline__ bool tri_finish_part(
    const double *Gin, const double *lamw, const double *Ug, const double *scp, int n, int k,
    int kw, double *lam_out, double *U_out, T *P, T *S, double *tail, int *ctl, double tau,
    double *U1) {
  extern __shared__ double lds[];
  const int ld = n | 1;
  double *Z = lds;             // n x ld (k columns)
  double *E = lds + n * ld;    // k x ld
  double *W = E + n * ld;      // n x ld: Z after the Newton-Schulz step
  __shared__ double s_lam[kTeNMax + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, c = e - i * k;
    Z[i * ld + c] = Ug[e];
  }
  if (tid < kw) s_lam[tid] = lamw[tid];
  if (tid == 0) s_bad = 0;
  __syncthreads();
  // kept eigenvalues at or above tau lambda_1: the first pass resolves them;
  // when some kept one is below, only those above enter the checks below and
  // the second pass (trunc_refine.hip) forms the factors
  int kc = k;
  if (ctl) {
    const double thr = tau * s_lam[0];
    kc = 0;
    while (kc < k && s_lam[kc] >= thr) ++kc;
    if (tau <= 0.0 || kc == 0) kc = k;
  }
  const int kg = (kc < k) ? kc : kw;  // eigenvalues whose gaps are checked
  if (wave == 0) {
    double mingap = 1e300;
    for (int w = lane; w + 1 < kg; w += 64) mingap = fmin(mingap, s_lam[w] - s_lam[w + 1]);
    mingap = wave_min(mingap);
    if (lane == 0 && !(mingap >= 1e-9)) s_bad = 1;
  }
  lds_gemm<true, false>(Z, ld, Z, ld, E, ld, kc, kc, n, 1.0, nullptr, 0, 0.0);
  __syncthreads();
  {
    double dev = 0.0;
    for (int e = tid; e < kc * kc; e += blockDim.x) {
      const int a = e / kc, b = e - a * kc;
      dev = fmax(dev, fabs(E[a * ld + b] - (a == b ? 1.0 : 0.0)));
    }
    dev = wave_max(dev);
    if (lane == 0 && !(dev <= 1e-6)) s_bad = 1;
  }
  __syncthreads();
  if (s_bad) return false;
  for (int e = tid; e < kc * kc; e += blockDim.x) {
    const int a = e / kc, b = e - a * kc;
    E[a * ld + b] = (a == b ? 1.5 : 0.0) - 0.5 * E[a * ld + b];
  }
  __syncthreads();
  lds_gemm<false, false>(Z, ld, E, ld, W, ld, n, kc, kc);
  for (int e = tid; e < n * (k - kc); e += blockDim.x) {  // columns past kc as they are
    const int i = e / (k - kc), c = kc + (e - i * (k - kc));
    W[i * ld + c] = Z[i * ld + c];
  }
  __syncthreads();
  Z = W;
  if (ctl && tid == 0) {
    ctl[0] = kc < k ? 1 : 0;
    ctl[1] = kc;
    ctl[2] = 0;
    ctl[3] = k;
  }
  // the outputs below read Z; the basis of the second pass is built after
  const bool second = ctl && kc < k;
  const double inv_sc = 1.0 / *scp;
  const double l0 = fmax(s_lam[0] * inv_sc, 0.0);
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, j = e - i * k;
    const double u = Z[i * ld + j];
    const double lj = s_lam[j] * inv_sc;
    const double sq = lj > 0.0 ? sqrt_f64(lj) : 0.0;
    U_out[e] = u;
    P[i * k + j] = (T)(u * sq);
    S[j * n + i] = (T)((lj > 1e-13 * l0 && lj > 0.0) ? u * rcp_f64(sq) : 0.0);
  }
  if (tid < k) lam_out[tid] = s_lam[tid] * inv_sc;
  if (wave == 0) {
    double tr = 0.0, kept = 0.0;
    for (int i = lane; i < n; i += 64) tr += Gin[i * n + i];
    for (int i = lane; i < k; i += 64) kept += s_lam[i];
    tr = wave_sum(tr);
    kept = wave_sum(kept) * inv_sc;
    if (lane == 0) *tail = fmax(tr - kept, 0.0);
  }
  if (second) {
    __syncthreads();
    complement_basis(Z, ld, n, kc, E, lds, U1);  // lds: the Z before the Newton-Schulz step
  }
  return true;
}

// Kernel 3 with its fallback: when the tridiagonal solver flagged trouble
// (non-finite T, close eigenvalues, lost orthogonality) the same workgroup
// diagonalises G by cyclic Jacobi and forms the truncation factors from it;
// the flag then stays set.
template <typename T>
__device__ __forceinline__ void tri_finish_kernel_body(
    const double *Gin, const double *lamw, const double *Ug, const double *scp, int n, int k,
    int kw, double *lam_out, double *U_out, T *P, T *S, double *tail, int *flag, int force,
    int *ctl = nullptr, double tau = 0.0, double *U1 = nullptr) {
  if (!force && *flag == 0 &&
      tri_finish_part<T>(Gin, lamw, Ug, scp, n, k, kw, lam_out, U_out, P, S, tail, ctl, tau,
                         U1))
    return;
  __syncthreads();
  jacobi_eig_kernel_body(Gin, lam_out, U_out, n, nullptr, nullptr);
  __syncthreads();
  trunc_factors_kernel_body<T>(lam_out, U_out, n, k, P, S, tail, nullptr);
  __shared__ int s_second;
  if (threadIdx.x == 0) {
    *flag = 1;
    s_second = 0;
    if (ctl) {
      int w = 0;
      const double thr = tau * lam_out[0];
      while (w < k && lam_out[w] >= thr) ++w;
      ctl[0] = (tau > 0.0 && w > 0 && w < k) ? 1 : 0;
      ctl[1] = w;
      ctl[2] = 0;
      ctl[3] = n;
      s_second = ctl[0];
    }
  }
  __syncthreads();
  // the Jacobi eigenvectors are a full orthonormal basis already
  if (s_second)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) U1[e] = U_out[e];
}

template <typename T>
__global__ __launch_bounds__(kTeThreads) void tri_finish_kernel(
    const double *Gin, const double *lamw, const double *Ug, const double *scp, int n, int k,
    int kw, double *lam_out, double *U_out, T *P, T *S, double *tail, int *flag, int force,
    int *ctl, double tau, double *U1) {
  tri_finish_kernel_body<T>(Gin, lamw, Ug, scp, n, k, kw, lam_out, U_out, P, S, tail, flag,
                            force, ctl, tau, U1);
}

template <int NMAX>
__global__ __launch_bounds__(kTrThreads) void tri_reduce_group_kernel(const EigGroupDesc *tab) {
  const EigGroupDesc &e = tab[blockIdx.x];
  tri_reduce_body<NMAX>(e.G, e.n, e.d, e.e, e.sc, e.Vr, e.taus, e.flag);
}

template <int NMAX>
__global__ __launch_bounds__(64) void tri_vec_group_kernel(const EigGroupDesc *tab) {
  const EigGroupDesc &e = tab[blockIdx.y];
  if ((int)blockIdx.x >= e.kw) return;
  tri_vec_body<NMAX>(e.d, e.e, e.n, e.k, e.Vr, e.taus, e.lamw, e.Uz, e.flag, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kTeThreads) void tri_finish_group_kernel(const EigGroupDesc *tab, int force) {
  const EigGroupDesc &e = tab[blockIdx.x];
  tri_finish_kernel_body<T>(e.G, e.lamw, e.Uz, e.sc, e.n, e.k, e.kw, e.lam, e.U,
                            static_cast<T *>(e.P), static_cast<T *>(e.S), e.tail, e.flag, force);
}

}  // namespace

static int g_eig_mode = 0;  // 0 tridiagonal solver (Jacobi on its failure), 1 Jacobi always

void eig_set_mode(int mode) { g_eig_mode = mode; }

// dynamic LDS of the finish kernel: Z, E and W of kernel 3, or G and V of
// the Jacobi fallback, whichever is larger
static size_t finish_lds(int n) {
  const int ld = n | 1, np = (n + 1) & ~1;
  return sizeof(double) * std::max<size_t>(3 * (size_t)n * ld, 2 * (size_t)np * (np + 1));
}

template <typename T>
int eig_trunc(const double *G, int64_t n, int64_t k, double *lam, double *U, T *P, T *S,
              double *tail, int *flag, double *scratch, hipStream_t s, int *ctl, double tau,
              double *U1) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "eigenproblem larger than the limit");
  if (k < 1 || k > n) return fail(TT_EINVAL, "truncation rank out of range");
  if (n <= kTeNMax) {
    const int kw = (int)std::min<int64_t>(k + 1, n);
    // scratch: d (n), e (n), sc (1), Vr (n*n), taus (n), lamw (n+1), U (n*k)
    double *d = scratch, *e = d + n, *sc = e + n, *Vr = sc + 1, *taus = Vr + n * n;
    double *lamw = taus + n, *Uz = lamw + n + 1;
    static bool attr_set = false;
    if (!attr_set) {
      TTR_HIP(hipFuncSetAttribute((const void *)tri_finish_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
      attr_set = true;
    }
    if (n <= 64)
      hipLaunchKernelGGL(tri_reduce_kernel<64>, dim3(1), dim3(kTrThreads), 0, s, G, (int)n, d, e,
                         sc, Vr, taus, flag);
    else
      hipLaunchKernelGGL(tri_reduce_kernel<80>, dim3(1), dim3(kTrThreads), 0, s, G, (int)n, d, e,
                         sc, Vr, taus, flag);
    TTR_HIP(hipGetLastError());
    if (n <= 64)
      hipLaunchKernelGGL(tri_vec_kernel<64>, dim3(kw), dim3(64), 0, s, d, e, (int)n, (int)k, Vr,
                         taus, lamw, Uz, flag);
    else
      hipLaunchKernelGGL(tri_vec_kernel<80>, dim3(kw), dim3(64), 0, s, d, e, (int)n, (int)k, Vr,
                         taus, lamw, Uz, flag);
    TTR_HIP(hipGetLastError());
    hipLaunchKernelGGL((tri_finish_kernel<T>), dim3(1), dim3(kTeThreads), finish_lds((int)n), s, G,
                       lamw, Uz, sc, (int)n, (int)k, kw, lam, U, P, S, tail, flag, g_eig_mode,
                       ctl, tau, U1);
    TTR_HIP(hipGetLastError());
    return TT_OK;
  }
  TTR_TRY(sym_eig(G, lam, U, n, s, nullptr, nullptr));
  if (ctl) TTR_TRY(trunc_refine_ctl(lam, U, n, k, tau, ctl, U1, s));
  return trunc_factors<T>(lam, U, n, k, P, S, tail, s, nullptr);
}

size_t eig_trunc_scratch(int64_t n, int64_t k) { return (size_t)(4 * n + 2 + n * n + n * k); }

template int eig_trunc<double>(const double *, int64_t, int64_t, double *, double *, double *,
                               double *, double *, int *, double *, hipStream_t, int *, double,
                               double *);
template int eig_trunc<float>(const double *, int64_t, int64_t, double *, double *, float *,
                              float *, double *, int *, double *, hipStream_t, int *, double,
                              double *);

bool eig_group_desc(const double *G, int64_t n, int64_t k, double *lam, double *U, void *P,
                    void *S, double *tail, int *flag, double *scratch, EigGroupDesc *d) {
  if (n > kTeNMax) return false;
  d->G = G;
  d->n = (int)n;
  d->k = (int)k;
  d->kw = (int)std::min<int64_t>(k + 1, n);
  d->d = scratch;
  d->e = d->d + n;
  d->sc = d->e + n;
  d->Vr = d->sc + 1;
  d->taus = d->Vr + n * n;
  d->lamw = d->taus + n;
  d->Uz = d->lamw + n + 1;
  d->lam = lam;
  d->U = U;
  d->P = P;
  d->S = S;
  d->tail = tail;
  d->flag = flag;
  return true;
}

template <typename T>
int eig_trunc_group(const EigGroupDesc *d_tab, int count, int nmax, int kwmax, hipStream_t s) {
  if (count <= 0) return TT_OK;
  if (nmax > kTeNMax) return fail(TT_EUNSUPPORTED, "grouped eigenproblem larger than the limit");
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)tri_finish_group_kernel<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
    attr_set = true;
  }
  if (nmax <= 64)
    hipLaunchKernelGGL(tri_reduce_group_kernel<64>, dim3(count), dim3(kTrThreads), 0, s, d_tab);
  else
    hipLaunchKernelGGL(tri_reduce_group_kernel<80>, dim3(count), dim3(kTrThreads), 0, s, d_tab);
  TTR_HIP(hipGetLastError());
  if (nmax <= 64)
    hipLaunchKernelGGL(tri_vec_group_kernel<64>, dim3(kwmax, count), dim3(64), 0, s, d_tab);
  else
    hipLaunchKernelGGL(tri_vec_group_kernel<80>, dim3(kwmax, count), dim3(64), 0, s, d_tab);
  TTR_HIP(hipGetLastError());
  hipLaunchKernelGGL((tri_finish_group_kernel<T>), dim3(count), dim3(kTeThreads), finish_lds(nmax),
                     s, d_tab, g_eig_mode);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}
template int eig_trunc_group<double>(const EigGroupDesc *, int, int, int, hipStream_t);
template int eig_trunc_group<float>(const EigGroupDesc *, int, int, int, hipStream_t);

}  // namespace ttr
