// Blocked Cholesky factorisation with the inverse of its factor, in one
// workgroup, shared by the thin QR (CholeskyQR passes) and the second pass
// of the truncation.
#pragma once
#include "fastmath.h"
#include "wave.h"

namespace ttr {
namespace {

// Upper Cholesky G = R^T R of the n x n FP64 matrix G (row-major,
// n <= NMAX), then Rinv = R^{-1} (upper triangular, row-major; with FP32
// storage also rounded to Rinv_f), by one workgroup of four wavefronts.
//
// Right-looking elimination on the augmented rows [G | I]: row j scaled by
// 1/sqrt(d_j) (d_j its current diagonal entry) is row j of R in its left part,
// and R[j][i] times it is subtracted from every row i > j; the left block
// ends as R and the right block as R^{-T} (the same row operations turn G
// into R = R^{-T} G), so Rinv is the transpose of the right block.  Padded
// rows and columns (n <= i < NMAX) hold the identity, which factors to
// itself without touching the rest.
//
// Blocked by panels of four columns: [G | I] lives in the accumulator layout
// of the f64 MFMA (16 x 16 blocks; block row I on wavefront I % 4; in a block
// lane (r, q) register jj holds row q + 4 jj, column r), so the four rows of
// a panel are register jj0 of the four lane groups q = 0..3 of one
// wavefront, which writes them to LDS as they stand.  After one barrier
// every lane factors the 4 x 4 diagonal block in registers (the same
// pivots, in the same order, as the unblocked elimination) and forms
// L^-1 (L = R4^T), whose row q turns the four raw rows into the final row
// q of the panel at any column; the owner keeps those rows, and every
// wavefront applies the rank-4 update to its rows below the panel with one
// MFMA per live 16 x 16 block (A: minus the panel's entries in the rows' own
// columns, B: the panel rows).  One barrier per panel instead of one per
// column; the LDS panel buffer alternates, so a panel is never overwritten
// while it is read.
//
// A pivot d_j that is not finite or not above piv_rel (1e-14) of the
// original diagonal entry raises the flag (or_flag = 0: flag overwritten,
// else or-ed; flag may be null) and is replaced by the original diagonal (1
// if that is not positive) so that the results stay finite.  With nullmask
// (null mode, the second truncation pass) a pivot not above dnull marks its
// direction instead (nullmask[j] = 1).  NW wavefronts (4; 8 or 16 in the
// one-workgroup kernels of the rescue and the second truncation pass) share
// the block rows.
//
// The second pass of CholeskyQR2 (or_flag = 1) factors G = Q1^T Q1 = I + E
// with E of the order of cond(Y)^2 u.  When max |E_ij| <= tol the factor is
// taken to first order, R = I + F with F = triu(E) - diag(E)/2 (then
// R^T R = I + E + F^T F), and R^{-1} = I - F; both drop terms of order
// |E|^2 <= (n tol)^2, so Q = Q1 (I - F) agrees with the exact CholeskyQR2
// factor to rounding: tol = 2^-30 with FP64 storage ((96 tol)^2 < 1e-14),
// 2^-17 with FP32 storage (Rinv_f given; (96 tol)^2 < 7e-7, about ten FP32
// roundings).  Larger E takes the factorisation below.
constexpr int kCholThreads = 256;
constexpr double kNearIdentity = 0x1p-30, kNearIdentityF32 = 0x1p-17;
typedef double chol_d4 __attribute__((ext_vector_type(4)));

template <int NMAX, int NW = 4>
__device__ __forceinline__ int chol_inv_kernel_body(const double *G, double *Rinv,
                                                    float *Rinv_f, int n, int *flag,
                                                    int or_flag, double sh = 0.0,
                                                    int mark = 0, double piv_rel = 1e-14,
                                                    int *nullmask = nullptr, double dnull = 0.0) {
  constexpr int NT = 64 * NW;               // threads
  constexpr int NRB = NMAX / 16;            // block rows
  constexpr int NCB = 2 * NRB;              // block columns of [G | I]
  constexpr int NSL = (NRB + NW - 1) / NW;  // block rows per wavefront
  static_assert(NMAX % 16 == 0, "rows in blocks of 16");
  __shared__ double s_pan[2][4][2 * NMAX];  // the scaled rows of a panel
  __shared__ double s_d0[NMAX];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;

  if (or_flag) {
    // second pass: first-order factor when G is within 2^-30 of I
    // a thread's entries (rows wave + NW t, columns lane + 64 u) are loaded
    // together (addresses clamped into G, entries past n dropped after the
    // load) and kept for the factor below
    constexpr int NRW = (NMAX + NW - 1) / NW, NCU = (NMAX + 63) / 64;
    __shared__ double s_emax[NW];
    double gv[NRW][NCU];
#pragma unroll
    for (int t = 0; t < NRW; ++t)
#pragma unroll
      for (int u = 0; u < NCU; ++u) {
        const int i = min(wave + NW * t, n - 1), c = min(lane + 64 * u, n - 1);
        gv[t][u] = G[i * n + c];
      }
    double em = 0.0;
#pragma unroll
    for (int t = 0; t < NRW; ++t)
#pragma unroll
      for (int u = 0; u < NCU; ++u) {
        const int i = wave + NW * t, c = lane + 64 * u;
        if (i < n && c < n) em = fmax(em, fabs(gv[t][u] - (i == c ? 1.0 : 0.0)));
      }
    em = fmax(em, __shfl_xor(em, 32));
    em = fmax(em, __shfl_xor(em, 16));
    em = fmax(em, __shfl_xor(em, 8));
    em = fmax(em, __shfl_xor(em, 4));
    em = fmax(em, __shfl_xor(em, 2));
    em = fmax(em, __shfl_xor(em, 1));
    if (lane == 0) s_emax[wave] = em;
    __syncthreads();
    double emax = s_emax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) emax = fmax(emax, s_emax[w]);
    if (emax <= (Rinv_f ? kNearIdentityF32 : kNearIdentity)) {  // also false for NaN
#pragma unroll
      for (int t = 0; t < NRW; ++t)
#pragma unroll
        for (int u = 0; u < NCU; ++u) {
          const int i = wave + NW * t, c = lane + 64 * u;
          if (i >= n || c >= n) continue;
          const int e = i * n + c;
          const double g = gv[t][u];
          const double x = (i == c) ? 1.0 - 0.5 * (g - 1.0) : ((i < c) ? -g : 0.0);
          Rinv[e] = x;
          if (Rinv_f) Rinv_f[e] = (float)x;
        }
      return 0;
    }
  }
  // sh: shift added to the diagonal (shifted CholeskyQR), 0 otherwise.
  // The lower-triangle entries G(max(i, c), min(i, c)) of a thread's part of
  // the left block columns are loaded first, all together (indices clamped
  // into G; entries outside the n x n matrix are not used).
  double gl[NSL][NRB][4];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl)
#pragma unroll
    for (int J = 0; J < NRB; ++J)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = 16 * (wave + NW * sl) + q + 4 * jj, c = 16 * J + r;
        const int hi = min(max(i, c), n - 1), lo = min(min(i, c), n - 1);
        gl[sl][J][jj] = G[hi * n + lo];
      }
  chol_d4 X[NSL][NCB];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    const int I = wave + NW * sl;
#pragma unroll
    for (int J = 0; J < NCB; ++J) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = 16 * I + q + 4 * jj, c = 16 * J + r;
        double v = 0.0;
        if (I < NRB) {
          if (J < NRB) {
            if (i < n && c < n) v = gl[sl][J][jj] + (i == c ? sh : 0.0);
            else if (i == c) v = 1.0;
          } else {
            v = (c - NMAX == i) ? 1.0 : 0.0;
          }
        }
        X[sl][J][jj] = v;
      }
    }
  }
  for (int i = tid; i < NMAX; i += NT) s_d0[i] = (i < n) ? G[i * n + i] + sh : 1.0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  int bad = 0;

  static_for<0, NMAX / 4>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    constexpr int j0 = 4 * p, I0 = j0 / 16, w0 = I0 % NW, sl0 = I0 / NW, jj0 = (j0 % 16) / 4;
    constexpr int buf = p & 1;
    // live block columns: left part from I0 on, right part up to column j0 + 3
    constexpr int JR = NRB + (j0 + 3) / 16;
    if (j0 >= n) return;
    // the owner publishes the four panel rows as they stand
    if (wave == w0) {
      static_for<I0, JR + 1>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int J = decltype(Jc)::value;
        s_pan[buf][q][16 * J + r] = X[sl0][J][jj0];
      });
    }
    __syncthreads();
    // every lane factors the 4 x 4 diagonal block D = R4^T R4 itself (the
    // unblocked pivots d_t = D_tt - sum_{s<t} R4_st^2) and forms the rows of
    // L^-1, L = R4^T, which turn the raw panel rows into rows of [R | R^-T]
    double R4[4][4], Li[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double d = s_pan[buf][t][j0 + t];
#pragma unroll
      for (int u = 0; u < t; ++u) d = fma(-R4[u][t], R4[u][t], d);
      const double d0 = s_d0[j0 + t];
      double rr, rt;  // 1 / sqrt(d), sqrt(d)
      if (nullmask) {
        // null mode: a pivot not above dnull is a direction with nothing
        // left; its row of R is made 1e300 on the diagonal and ~0 elsewhere,
        // its row of R^-T ~0, so that it updates nothing below
        const bool nul = (j0 + t < n) && !(d > dnull);
        if (tid == 0 && j0 + t < n) nullmask[j0 + t] = nul ? 1 : 0;
        rr = nul ? 1e-300 : rsq_f64(d);
        rt = nul ? 1e300 : d * rr;
      } else {
        if (!(d > piv_rel * d0) || !(d0 > 0.0) || !isfinite(d)) {
          d = (d0 > 0.0 && isfinite(d0)) ? d0 : 1.0;
          bad = 1;
        }
        rr = rsq_f64(d);
        rt = d * rr;
      }
      R4[t][t] = rt;
#pragma unroll
      for (int c = t + 1; c < 4; ++c) {
        double x = s_pan[buf][t][j0 + c];
#pragma unroll
        for (int u = 0; u < t; ++u) x = fma(-R4[u][t], R4[u][c], x);
        R4[t][c] = x * rr;
      }
      Li[t][t] = rr;
#pragma unroll
      for (int u = 0; u < t; ++u) {
        double x = 0.0;
#pragma unroll
        for (int v = u; v < t; ++v) x = fma(R4[v][t], Li[v][u], x);
        Li[t][u] = -rr * x;
      }
    }
    // this lane's row q of L^-1
    double cq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      cq[u] = (u > q) ? 0.0
                      : (q == 0 ? Li[0][u] : q == 1 ? Li[1][u] : q == 2 ? Li[2][u] : Li[3][u]);
    // final panel row q at column col (left-block entries left of the
    // diagonal are zero, the diagonal is sqrt(d))
    auto panel_at = [&](int col) -> double {
      double x = cq[0] * s_pan[buf][0][col];
#pragma unroll
      for (int u = 1; u < 4; ++u) x = fma(cq[u], s_pan[buf][u][col], x);
      return x;
    };
    const double rdiag = q == 0 ? R4[0][0] : q == 1 ? R4[1][1] : q == 2 ? R4[2][2] : R4[3][3];
    // row q of the final panel at this lane's column of every live block,
    // formed once for the owner's rows and the update's B operands
    double pv[NCB];
    static_for<I0, JR + 1>([&](auto Jc) __attribute__((always_inline)) {
      constexpr int J = decltype(Jc)::value;
      pv[J] = panel_at(16 * J + r);
    });
    if (wave == w0) {
      static_for<I0, JR + 1>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int J = decltype(Jc)::value;
        double x = pv[J];
        if constexpr (J < NRB) {
          const int c = 16 * J + r;
          if (c == j0 + q) x = rdiag;
          if (c < j0 + q) x = 0.0;
        }
        X[sl0][J][jj0] = x;
      });
    }
    // rank-4 update of the rows below the panel: X_IJ -= L_I P_J (lane (r, q)
    // gives A[r][q] = -P_q(row 16 I + r) and B[q][r] = P_q(16 J + r))
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      const int I = wave + NW * sl;
      if (I >= I0 && I < NRB) {
        const int row = 16 * I + r;
        const double a = (row > j0 + 3) ? -panel_at(row) : 0.0;
        static_for<I0, JR + 1>([&](auto Jc) __attribute__((always_inline)) {
          constexpr int J = decltype(Jc)::value;
          X[sl][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, pv[J], X[sl][J], 0, 0, 0);
        });
      }
    }
  });
  if (bad) s_bad = 1;
  // Rinv[c][i] = B[i][c] (right block, lower triangular)
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    const int I = wave + NW * sl;
    if (I < NRB) {
#pragma unroll
      for (int J = NRB; J < NCB; ++J) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = 16 * I + q + 4 * jj, c = 16 * (J - NRB) + r;
          if (i < n && c < n) {
            const double x = (c <= i) ? X[sl][J][jj] : 0.0;
            Rinv[(int64_t)c * n + i] = x;
            if (Rinv_f) Rinv_f[(int64_t)c * n + i] = (float)x;
          }
        }
      }
    }
  }
  __syncthreads();
  const int bad_all = s_bad;
  if (tid == 0 && flag) {
    if (or_flag) {
      // after a shifted first pass (bit 1) the third pass decides
      if (bad_all && !(*flag & 2)) *flag = *flag | 1;
    } else {
      *flag = bad_all | mark;
    }
  }
  return bad_all;
}

}  // namespace
}  // namespace ttr
