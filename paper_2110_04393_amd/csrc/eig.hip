// Symmetric eigendecomposition for the truncation step.
//
// The truncation of the left-orthogonal RtO output (section 3.2, remark after
// Algorithm 5; the mirror of the truncation loop of Algorithm 2) needs, at each bond, the
// leading singular triplets of H(X_n).  With G = H(X_n) H(X_n)^T = U s^2 U^T:
//   H(X_n) <- s^-1 U^T H(X_n),   X_{n-1} <- X_{n-1} x_3 (U s),
// which is the SVD truncation written with the Gram matrix (equal to it in
// exact arithmetic; singular values below about 1e-7 of the largest are
// resolved only to FP64 rounding of the Gram).
//
// G (n <= 96) is diagonalised by cyclic two-sided Jacobi in one workgroup
// with G and the accumulated rotations V resident in LDS.  Each round applies
// n/2 disjoint rotations at once (round-robin pairing): phase A computes the
// rotation of every pair, phase B updates every 2x2 block
// G[{p_k,q_k}][{p_m,q_m}] <- J_k^T G J_m and V[:, {p_m,q_m}] <- V J_m, with
// J = [[c, s], [-s, c]] chosen so that the (p, q) entry vanishes.
#include "tt_internal.h"

namespace ttr {
namespace {

constexpr int kEigThreads = 512;
constexpr int kMaxSweeps = 40;

__device__ inline void round_pair(int t, int k, int np, int &p, int &q) {
  const int m = np - 1;
  int a, b;
  if (k == 0) {
    a = m;
    b = t;
  } else {
    a = (t + k) % m;
    b = (t - k + m) % m;
  }
  p = min(a, b);
  q = max(a, b);
}

__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(const double *Gin, double *lam,
                                                                 double *Uout, int n) {
  extern __shared__ double lds[];
  const int np = (n + 1) & ~1;
  double *G = lds;              // np*np
  double *V = lds + np * np;    // np*np
  __shared__ double s_c[64], s_s[64];
  __shared__ int s_p[64], s_q[64];
  __shared__ int s_rot;
  __shared__ double s_scale;
  const int tid = threadIdx.x;
  for (int e = tid; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e - i * np;
    G[e] = (i < n && j < n) ? Gin[i * n + j] : 0.0;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double sc = 0.0;
    for (int i = 0; i < n; ++i) sc = fmax(sc, fabs(G[i * np + i]));
    s_scale = sc;
  }
  __syncthreads();
  const double floor_abs = 1e-20 * s_scale;
  const int npairs = np / 2;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int t = 0; t < np - 1; ++t) {
      if (tid < npairs) {
        int p, q;
        round_pair(t, tid, np, p, q);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = G[p * np + p], aqq = G[q * np + q], apq = G[p * np + q];
          const double thr = fmax(1e-15 * sqrt(fabs(app * aqq)), floor_abs);
          if (fabs(apq) > thr) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) /
                              (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
            c = 1.0 / sqrt(fma(tt, tt, 1.0));
            s = tt * c;
            atomicAdd(&s_rot, 1);
          }
        }
        s_c[tid] = c;
        s_s[tid] = s;
        s_p[tid] = p;
        s_q[tid] = q;
      }
      __syncthreads();
      // phase B: 2x2 blocks of G, then row pairs of V
      for (int e = tid; e < npairs * npairs; e += blockDim.x) {
        const int k = e / npairs, m = e - k * npairs;
        const double ck = s_c[k], sk = s_s[k], cm = s_c[m], sm = s_s[m];
        if (sk == 0.0 && sm == 0.0) continue;
        const int p = s_p[k], q = s_q[k], pp = s_p[m], qq = s_q[m];
        const double b00 = G[p * np + pp], b01 = G[p * np + qq];
        const double b10 = G[q * np + pp], b11 = G[q * np + qq];
        // B J_m
        const double x00 = cm * b00 - sm * b01, x01 = sm * b00 + cm * b01;
        const double x10 = cm * b10 - sm * b11, x11 = sm * b10 + cm * b11;
        // J_k^T (B J_m)
        G[p * np + pp] = ck * x00 - sk * x10;
        G[p * np + qq] = ck * x01 - sk * x11;
        G[q * np + pp] = sk * x00 + ck * x10;
        G[q * np + qq] = sk * x01 + ck * x11;
      }
      for (int e = tid; e < n * npairs; e += blockDim.x) {
        const int i = e / npairs, m = e - i * npairs;
        const double cm = s_c[m], sm = s_s[m];
        if (sm == 0.0) continue;
        const int pp = s_p[m], qq = s_q[m];
        const double vp = V[i * np + pp], vq = V[i * np + qq];
        V[i * np + pp] = cm * vp - sm * vq;
        V[i * np + qq] = sm * vp + cm * vq;
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
  // sort descending (stable by index)
  for (int i = tid; i < n; i += blockDim.x) {
    const double li = G[i * np + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = G[j * np + j];
      rank += (lj > li) || (lj == li && j < i);
    }
    lam[rank] = li;
    for (int r = 0; r < n; ++r) Uout[r * n + rank] = V[r * np + i];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void trunc_factors_kernel(const double *lam, const double *U,
                                                            int n, int k, T *P, T *S,
                                                            double *tail) {
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

int sym_eig(const double *G, double *lam, double *U, int64_t n, hipStream_t s) {
  if (n > TT_MAX_SKETCH_RANK) return fail(TT_EUNSUPPORTED, "eigenproblem larger than the limit");
  const int np = (int)((n + 1) & ~1);
  const size_t lds = 2 * sizeof(double) * (size_t)np * np;
  static bool attr_set = false;
  if (!attr_set) {
    TTR_HIP(hipFuncSetAttribute((const void *)jacobi_eig_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048));
    attr_set = true;
  }
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(kEigThreads), lds, s, G, lam, U, (int)n);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template <typename T>
int trunc_factors(const double *lam, const double *U, int64_t n, int64_t k, T *P, T *S,
                  double *tail, hipStream_t s) {
  hipLaunchKernelGGL((trunc_factors_kernel<T>), dim3(1), dim3(256), 0, s, lam, U, (int)n, (int)k,
                     P, S, tail);
  TTR_HIP(hipGetLastError());
  return TT_OK;
}

template int trunc_factors<double>(const double *, const double *, int64_t, int64_t, double *,
                                   double *, double *, hipStream_t);
template int trunc_factors<float>(const double *, const double *, int64_t, int64_t, float *,
                                  float *, double *, hipStream_t);

}  // namespace ttr
