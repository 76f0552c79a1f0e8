// Device bodies of the cyclic Jacobi eigensolver and of the truncation
// factors, shared by their own kernels and by the fused eigen-finish kernel
// (the Jacobi solve is the fallback of the tridiagonal solver).
#pragma once
#include "fastmath.h"
#include "tt_internal.h"

namespace ttr {
namespace {

constexpr int kEigThreads = 512;
constexpr int kMaxSweeps = 40;
constexpr int kMaxBlocksOwn = 5;   // 48*48 2x2 blocks over 512 threads
constexpr int kMaxVOwn = 9;        // 96*48 row pairs of V over 512 threads

// Pair k of round t in the round-robin ("circle") ordering of np indices:
// pair 0 = (np-1, t), pair k = ((t+k) mod (np-1), (t-k) mod (np-1)).
__device__ inline void round_pair(int t, int k, int np, int &p, int &q) {
  const int m = np - 1;
  int a, b;
  if (k == 0) {
    a = m;
    b = t;
  } else {
    a = t + k;
    if (a >= m) a -= m;
    b = t - k;
    if (b < 0) b += m;
  }
  p = min(a, b);
  q = max(a, b);
}

__device__ __forceinline__ void jacobi_eig_kernel_body(const double *Gin, double *lam,
                                                                 double *Uout, int n,
                                                                 int *info, const int *gate,
                                                                 bool relative = false) {
  if (gate && *gate == 0) return;
  extern __shared__ double lds[];
  const int np = (n + 1) & ~1;
  const int ld = np + 1;
  double *G = lds;             // np x ld
  double *V = lds + np * ld;   // np x ld
  __shared__ double s_c[48], s_s[48];
  __shared__ int s_p[48], s_q[48];
  __shared__ double s_offmax[48];
  __shared__ double s_scale;
  const int tid = threadIdx.x;
  const int npairs = np / 2;
  for (int e = tid; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e - i * np;
    G[i * ld + j] = (i < n && j < n) ? Gin[i * n + j] : 0.0;
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  // static ownership of 2x2 blocks (k, m) and of V row pairs (i, m)
  int bk[kMaxBlocksOwn], bm[kMaxBlocksOwn], vi[kMaxVOwn], vm[kMaxVOwn];
  int nb = 0, nv = 0;
  for (int e = tid; e < npairs * npairs && nb < kMaxBlocksOwn; e += blockDim.x) {
    bk[nb] = e / npairs;
    bm[nb] = e - bk[nb] * npairs;
    ++nb;
  }
  for (int e = tid; e < n * npairs && nv < kMaxVOwn; e += blockDim.x) {
    vi[nv] = e / npairs;
    vm[nv] = e - vi[nv] * npairs;
    ++nv;
  }
  __syncthreads();
  if (tid == 0) {
    double sc = 0.0;
    for (int i = 0; i < n; ++i) sc = fmax(sc, fabs(G[i * ld + i]));
    s_scale = sc;
  }
  __syncthreads();
  // A pair is rotated when apq^2 > tol^2 |app aqq| (relative test) and
  // |apq| > floor_abs: couplings at the rounding level of the largest diagonal
  // entry (about n u max|G_ii|, the error of the Gram itself) are left alone,
  // otherwise the relative test cannot be met for small diagonal entries.
  // With `relative` the floor is off: for a matrix whose entries carry their
  // own relative accuracy (the Gram of nearly orthogonal rows), every
  // coupling is rotated until the relative test holds.
  const double tol2 = 1e-30;
  const double floor_abs = relative ? 0.0 : 1.2e-16 * (double)n * s_scale;
  int sweeps = 0;
  double offmax = 0.0;  // per pair-lane: largest relative coupling seen this sweep
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    ++sweeps;
    offmax = 0.0;
    for (int t = 0; t < np - 1; ++t) {
      // phase A: one rotation per pair (lanes of the first wavefront)
      if (tid < npairs) {
        int p, q;
        round_pair(t, tid, np, p, q);
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double app = G[p * ld + p], aqq = G[q * ld + q], apq = G[p * ld + q];
          const double prod = fabs(app * aqq);
          const double a2 = apq * apq;
          if (a2 > tol2 * prod && fabs(apq) > floor_abs) {
            offmax = fmax(offmax, prod > 0.0 ? a2 / prod : 1.0);
            // theta = (aqq - app) / (2 apq); t = sign(theta) / (|theta| + sqrt(theta^2 + 1))
            const double theta = (aqq - app) * rcp_f64(2.0 * apq);
            const double at = fabs(theta);
            double tt;
            if (at > 1e150) {
              tt = 0.5 * rcp_f64(at);
            } else {
              const double h = fma(at, at, 1.0);
              tt = rcp_f64(at + sqrt_f64(h));
            }
            if (theta < 0.0) tt = -tt;
            c = rsq_f64(fma(tt, tt, 1.0));
            sn = tt * c;
          }
        }
        s_c[tid] = c;
        s_s[tid] = sn;
        s_p[tid] = p;
        s_q[tid] = q;
      }
      __syncthreads();
      // phase B: G[{p_k,q_k}][{p_m,q_m}] <- J_k^T G J_m and V[i][{p_m,q_m}] <- V J_m
#pragma unroll
      for (int o = 0; o < kMaxBlocksOwn; ++o) {
        if (o >= nb) break;
        const int k = bk[o], m = bm[o];
        const double ck = s_c[k], sk = s_s[k], cm = s_c[m], sm = s_s[m];
        if (sk == 0.0 && sm == 0.0) continue;
        const int p = s_p[k], q = s_q[k], pp = s_p[m], qq = s_q[m];
        const double b00 = G[p * ld + pp], b01 = G[p * ld + qq];
        const double b10 = G[q * ld + pp], b11 = G[q * ld + qq];
        const double x00 = cm * b00 - sm * b01, x01 = sm * b00 + cm * b01;
        const double x10 = cm * b10 - sm * b11, x11 = sm * b10 + cm * b11;
        G[p * ld + pp] = ck * x00 - sk * x10;
        G[p * ld + qq] = ck * x01 - sk * x11;
        G[q * ld + pp] = sk * x00 + ck * x10;
        G[q * ld + qq] = sk * x01 + ck * x11;
      }
#pragma unroll
      for (int o = 0; o < kMaxVOwn; ++o) {
        if (o >= nv) break;
        const int i = vi[o], m = vm[o];
        const double cm = s_c[m], sm = s_s[m];
        if (sm == 0.0) continue;
        const int pp = s_p[m], qq = s_q[m];
        const double vp = V[i * ld + pp], vq = V[i * ld + qq];
        V[i * ld + pp] = cm * vp - sm * vq;
        V[i * ld + qq] = sm * vp + cm * vq;
      }
      __syncthreads();
    }
    // quadratic convergence: once the largest relative coupling rotated in a
    // sweep is below 1e-8, what is left after it is at the 1e-16 level.
    if (tid < npairs) s_offmax[tid] = offmax;
    __syncthreads();
    double mx = 0.0;
    for (int k = 0; k < npairs; ++k) mx = fmax(mx, s_offmax[k]);
    __syncthreads();
    if (mx <= 1e-16) break;  // (relative coupling)^2 <= 1e-16
  }
  // sort descending (ties by index)
  for (int i = tid; i < n; i += blockDim.x) {
    const double li = G[i * ld + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = G[j * ld + j];
      rank += (lj > li) || (lj == li && j < i);
    }
    lam[rank] = li;
    for (int r = 0; r < n; ++r) Uout[r * n + rank] = V[r * ld + i];
  }
  if (tid == 0 && info) *info = sweeps;
  (void)offmax;
}

template <typename T>
__device__ __forceinline__ void trunc_factors_kernel_body(const double *lam, const double *U,
                                                            int n, int k, T *P, T *S,
                                                            double *tail, const int *gate) {
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  const double l0 = fmax(lam[0], 0.0);
  const double thr = 1e-13 * l0;
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int i = e / k, j = e - i * k;
    const double lj = lam[j];
    const double sq = lj > 0.0 ? sqrt(lj) : 0.0;
    P[i * k + j] = (T)(U[i * n + j] * sq);
    S[j * n + i] = (T)((lj > thr && lj > 0.0) ? U[i * n + j] / sq : 0.0);
  }
  if (tid == 0) {
    double t = 0.0;
    for (int j = k; j < n; ++j) t += fmax(lam[j], 0.0);
    *tail = t;
  }
}

}  // namespace
}  // namespace ttr
